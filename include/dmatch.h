/*
 * dmatch.h - C ABI of the MI355X (gfx950) library for discrete-continuous dense matching.
 *
 * Method: Shekhovtsov, Reinbacher, Graber, Pock, "Solving Dense Image Matching in
 * Real-Time using Discrete-Continuous Optimization" (CVWW 2016).
 *
 * Conventions shared by every entry point
 *   - Every array pointer is a DEVICE pointer (e.g. the storage of a torch tensor on
 *     the GPU) unless stated otherwise; parameter structs are HOST pointers.
 *   - Images and per-pixel arrays are row-major [H][W]: pixel (x, y) at y*W + x.
 *   - Volumes are label-major [H][W][K]: label k of pixel (x, y) at (y*W + x)*K + k.
 *   - Edge arrays: w_h[H][W-1] holds the edge between (x, y) and (x+1, y) at
 *     y*(W-1) + x; w_v[H-1][W] holds the edge between (x, y) and (x, y+1) at y*W + x.
 *     Edge weights must be finite and >= 0.
 *   - The caller owns every buffer.  Calls that need scratch memory take a caller
 *     workspace whose size is given by the matching *_workspace() query; the library
 *     allocates no device memory in these calls.
 *   - Work is enqueued on `hip_stream` (a hipStream_t, NULL = the null stream) and is
 *     asynchronous: outputs are valid once the stream has completed.
 *   - Return value: DM_OK or a negative dm_status.  Arguments are validated on the
 *     host before anything is enqueued; on a validation error nothing is launched and
 *     no output is touched.  A launch failure, or an asynchronous fault left by an
 *     earlier call, is returned as DM_ERR_HIP.  No C++ exception crosses this ABI.
 *     dm_last_error_message() gives a thread-local description of the last error.
 *   - Non-finite values (NaN/Inf) in cost volumes or images give unspecified results.
 */
#ifndef DMATCH_H
#define DMATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DM_OK = 0,
    DM_ERR_NULL = -1,        /* a required pointer is NULL                       */
    DM_ERR_SHAPE = -2,       /* W, H or K out of range                           */
    DM_ERR_PARAM = -3,       /* a parameter value is out of range                */
    DM_ERR_DTYPE = -4,       /* unknown dm_dtype                                 */
    DM_ERR_WORKSPACE = -5,   /* workspace NULL or smaller than the size query    */
    DM_ERR_UNSUPPORTED = -6, /* valid but not compiled into this library        */
    DM_ERR_HIP = -7          /* HIP runtime error (launch or asynchronous fault) */
} dm_status;

typedef enum { DM_F32 = 0, DM_F16 = 1 } dm_dtype;   /* storage type of the cost volume */

typedef enum { DM_MINORANT_ITERATIVE = 0, DM_MINORANT_NAIVE = 1, DM_MINORANT_HIERARCHICAL = 2 } dm_minorant;

/* Grid of W x H pixels with K labels; 1 <= W, H <= 16384, 1 <= K <= 256, and one FP32
 * volume (W*H*K*4 bytes) at most 0xFE000000 bytes: the kernels address volumes with
 * 32-bit byte offsets.  Larger shapes fail with DM_ERR_SHAPE. */
typedef struct { int W, H, K; } dm_shape;

/* ---------------------------------------------------------------------------------
 * Cost volume (paper Sec. 2.2 "Stereo": the data term sampled at every label; the
 * paper's own data term is Census + Hamming, Sec. 3.1 - this library provides a
 * truncated SAD of the same role).
 *
 *   e(x,y,d)     = |I_L(x,y) - I_R(x-d,y)|  if x-d >= 0, else trunc
 *   cost[y][x][d] = min(trunc, mean of e over the window x.+-r, y.+-r clamped to the image)
 *   w_h[y][x]    = lambda_pw * exp(-|I_L(x+1,y) - I_L(x,y)| / contrast_sigma)
 *   w_v[y][x]    = lambda_pw * exp(-|I_L(x,y+1) - I_L(x,y)| / contrast_sigma)
 * (edge strengths lower across image edges, Sec. 2.1 below eq. regularizer-form).
 *
 * I_left, I_right: [H][W] float32.  cost_out: [H][W][K] of out_dtype (FP16 values are
 * the FP32 result rounded to nearest even).  w_h / w_v may be NULL (not computed).
 * window: odd, 1..15.  trunc > 0, lambda_pw >= 0, contrast_sigma > 0.
 * ------------------------------------------------------------------------------- */
typedef struct { int window; float trunc; float lambda_pw; float contrast_sigma; } dm_cost_params;

int dm_build_cost_volume(const float* I_left, const float* I_right, dm_shape s,
                         const dm_cost_params* p, dm_dtype out_dtype, void* cost_out,
                         float* w_h, float* w_v, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Census + Hamming cost volume: the paper's data term (Sec. 3.1 "Stereo
 * Reconstruction": the Census transform of each image on a small patch, compared by
 * the pixel-wise Hamming distance).  The paper fixes neither the patch nor the
 * comparison; here
 *
 *   census(I)(x,y) = bits [I(q_b) < I(x,y)] over the non-centre positions q_b of the
 *                    window x.+-r, y.+-r (raster order, dy outer; clamped to the
 *                    image), n = (2r+1)^2 - 1 bits
 *   view DM_VIEW_LEFT:  cost[y][x][d] = min(trunc, H(cL(x,y), cR(x-d,y)) / n) if x-d >= 0
 *   view DM_VIEW_RIGHT: cost[y][x][d] = min(trunc, H(cR(x,y), cL(x+d,y)) / n) if x+d < W
 *   (H = number of differing bits; a match outside the image costs trunc)
 *
 * Each value is the correctly rounded quotient, stored as out_dtype (FP16 rounded to
 * nearest even).  w_h / w_v (may be NULL) are the contrast weights of dm_build_cost_volume
 * computed from the view's own image (I_left for the left view, I_right for the right).
 * p->window: 3, 5 or 7; 0 < p->trunc <= 1 (1: no truncation); lambda_pw >= 0,
 * contrast_sigma > 0.  Arrays are device memory owned by the caller; the call only
 * enqueues work on hip_stream.  Errors: DM_ERR_NULL, DM_ERR_SHAPE, DM_ERR_DTYPE,
 * DM_ERR_PARAM (window, trunc, view), DM_ERR_HIP (pending or launch error).
 * ------------------------------------------------------------------------------- */
enum { DM_VIEW_LEFT = 0, DM_VIEW_RIGHT = 1 };
int dm_build_cost_volume_census(const float* I_left, const float* I_right, dm_shape s,
                                const dm_cost_params* p, int view, dm_dtype out_dtype,
                                void* cost_out, float* w_h, float* w_v, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Left-right consistency check (the two-sided check of Sec. 4.1 that removes the
 * outliers of one view; Table tab:timing notes that it doubles the time, since the
 * right view is solved as well).
 *
 *   r = round half up of u_left(x,y);  x' = x - r
 *   u_out(x,y) = u_left(x,y)  if 0 <= x' < W and |u_left(x,y) - u_right(x',y)| <= max_diff
 *              = invalid      otherwise
 *
 * u_left, u_right, u_out: [H][W] float32 device arrays (disparities of the left view
 * and of the right view, the latter as produced from the DM_VIEW_RIGHT cost volume),
 * owned by the caller; u_out must not alias the inputs.  The rounding is exact; the
 * difference and its comparison are FP32.  W <= 2^24, W*H <= 2^31, max_diff >= 0.
 * Errors: DM_ERR_NULL, DM_ERR_SHAPE, DM_ERR_PARAM, DM_ERR_HIP.
 * ------------------------------------------------------------------------------- */
int dm_lr_check(const float* u_left, const float* u_right, int W, int H, float max_diff,
                float invalid, float* u_out, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Discrete stage: Dual_MM (paper Sec. 2.3, Alg. Dual_MM; minorants App. A.3).
 *
 * Energy (Sec. 2.2, eq. energy-pairwise):
 *   E(x) = sum_i cost_i(x_i) + sum_h w_h rho(x_i - x_j) + sum_v w_v rho(x_i - x_j),
 *   rho(t) = min(|t|, trunc_T)    (truncated linear; Potts for trunc_T = 1).
 * Decomposition: horizontal chains F with unaries cost - lambda and vertical chains G
 * with unaries lambda (lambda = dual_inout).  One dual iteration = a horizontal
 * half-step (each row hands its minorant to G: lambda += h) followed by a vertical
 * half-step (each column hands its minorant to F: lambda -= h).
 * Minorant DM_MINORANT_ITERATIVE: App. A.3.2 Alg. Iterative Minorant with max_pass
 * directional passes (forward first, then alternating) and steps gamma[0..max_pass-1];
 * gamma[max_pass-1] must be 1 (maximal minorant).  DM_MINORANT_NAIVE: normalized
 * min-marginals divided by the chain length (Sec. 2.3, App. A.1).
 * DM_MINORANT_HIERARCHICAL: App. A.3.3 (Alg. Handshake): every chain is cut in its
 * middle (the left part holding half of the nodes, rounded down), a Handshake over the
 * cut edge passes half of the min-marginal at its left node to the right part and
 * bounces back what cannot be passed, and each part is cut again down to single nodes;
 * node k's minorant is its unary plus the two Handshake messages it received, minus
 * its minimum.  Forward only (keep_checkpoints must be 0, else DM_ERR_UNSUPPORTED; no
 * batched plans, no tile autotuning); the chain tiles then apply to the final pass
 * only, the half-steps run one workgroup of one or four waves per chain and need a
 * second message volume in the workspace (included in dm_solve_discrete_workspace).
 *
 * Outputs after the last half-step:
 *   labels_out  [H][W] int32: argmin over k of the normalized row min-marginals of F
 *               (lowest k on exact ties).  May be NULL.
 *   minmarg_out [H][W][K] float32: those normalized min-marginals.  May be NULL.
 *   dual_inout  [H][W][K] float32: lambda.  Read as the starting point if warm_start,
 *               else overwritten with 0 first; holds the final lambda.  Required.
 *   bounds_out  device double[2] = {LB, E(labels)}; LB = min F + min G (eq. DD-dual).
 *               May be NULL.
 *   lb_trace_out device double[number of half-steps]: LB after each half-step.  May be NULL.
 * Numerics: FP32 state (lambda, messages), cost read as FP32 or FP16 and widened to
 * FP32; messages are renormalised to minimum 0 at every step; LB/E accumulate in FP64
 * in a fixed order (results are run-to-run deterministic).
 * ------------------------------------------------------------------------------- */
typedef struct {
    int   n_iters;          /* dual iterations (>= 0)                                   */
    int   n_half_steps;     /* > 0 overrides 2*n_iters (odd = ends after a horizontal)  */
    int   trunc_T;          /* truncation of rho, >= 1                                  */
    int   minorant;         /* dm_minorant                                              */
    int   max_pass;         /* 1..8 (iterative minorant)                                */
    float gamma[8];         /* each in (0, 1]; gamma[max_pass-1] == 1                   */
    int   warm_start;       /* 0: lambda := 0 first; 1: start from dual_inout           */
    int   tile_lanes;       /* row chains: 0 = automatic; else lanes per chain (4..64)  */
    int   labels_per_lane;  /* row chains: 0 = automatic; else with tile_lanes*lpl >= K */
    int   tile_lanes_v;     /* column chains: 0 = same as rows (see dm_autotune_tiles)  */
    int   labels_per_lane_v;
    int   keep_checkpoints; /* for dm_solve_discrete_backward (the size query includes
                               what is kept):
                               0: nothing kept;
                               1: the dual before every half-step (one FP32 volume per
                                  half-step; the backward recomputes the messages);
                               2: also what the backward would recompute (P = update
                                  passes): with selection tapes (below) every pass's tape
                                  (P + 1 tapes of W*H*lanes*ceil(lpl/4)*4 bytes, lanes x
                                  lpl the larger family tile); otherwise every pass's
                                  messages and the duals between passes (2*P volumes)  */
    int   recompute_selections; /* 0: the backward reads selection tapes - which operand
                               each min of a message took and each node's argmins,
                               one byte per label and pass, written by the recompute
                               (or, with keep_checkpoints 2, the forward) - whenever
                               the truncation reaches at most one lane across in both
                               families' tiles (trunc_T - 1 <= labels per lane) and a
                               tape fits 4 GiB; 1: the backward always recomputes the
                               selections from the forward's values (same results)   */
} dm_discrete_params;

size_t dm_solve_discrete_workspace(dm_shape s, dm_dtype cost_dtype, const dm_discrete_params* p);

int dm_solve_discrete(const void* cost, dm_dtype cost_dtype, const float* w_h, const float* w_v,
                      dm_shape s, const dm_discrete_params* p,
                      int32_t* labels_out, float* minmarg_out, float* dual_inout,
                      double* bounds_out, double* lb_trace_out,
                      void* workspace, size_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid allocation): dm_solve_discrete with the same arguments and
 * results, but without a workspace.  The scratch memory lives in a library-owned device
 * array of dm_solve_discrete_noalloc_limit() bytes (256 MiB) per GPU, held from the first
 * call on that GPU until the process ends; this call allocates nothing.  Problems whose
 * dm_solve_discrete_workspace() exceeds the limit fail with DM_ERR_WORKSPACE (e.g. K = 128
 * fits up to about 640 x 480 with keep_checkpoints = 0).  All calls on one GPU share the
 * array: calls that overlap in time on the same GPU race, so the caller serialises them. */
size_t dm_solve_discrete_noalloc_limit(void);
int dm_solve_discrete_noalloc(const void* cost, dm_dtype cost_dtype, const float* w_h, const float* w_v,
                              dm_shape s, const dm_discrete_params* p,
                              int32_t* labels_out, float* minmarg_out, float* dual_inout,
                              double* bounds_out, double* lb_trace_out, void* hip_stream);

/* The tile used when p->tile_lanes is 0: the compiled (lanes per chain, labels per lane)
 * tile with the fewest idle label slots for K labels (more lanes on ties).  Host only;
 * returns DM_ERR_SHAPE for K outside [1, 256], DM_ERR_NULL for null outputs. */
int dm_default_tile(int K, int* tile_lanes, int* labels_per_lane);

/* Autotuner: measures every compiled (lanes per chain, labels per lane) tile on one
 * half-step of a synthetic instance of shape s (row and column chains separately) and
 * writes the fastest into p->tile_lanes / labels_per_lane (rows) and tile_lanes_v /
 * labels_per_lane_v (columns).  Allocates and frees scratch device memory (unlike the
 * solver calls); synchronises hip_stream; results are cached for the process per
 * (W, H, K, cost dtype, minorant, max_pass). */
int dm_autotune_tiles(dm_shape s, dm_dtype cost_dtype, dm_discrete_params* p, void* hip_stream);

/* Adjoint of dm_solve_discrete (reverse mode; the paper gives no derivative - this is
 * the exact derivative of the piecewise-linear Dual_MM map as computed: minimisations
 * route the adjoint to the selected candidate, lowest label on exact ties).
 * Loss inputs: grad_minmarg [H][W][K] = dL/d(normalized row min-marginals) (may be NULL)
 * and grad_bounds, a device double[2] = {dL/dLB, dL/dE} matching bounds_out of the forward
 * (may be NULL: both 0; it is read on the device, so the call never waits for it).
 * E(labels) depends on the cost and the weights only through its terms at the output
 * labeling (the labels are piecewise constant): dE/dcost is the one-hot of the labels and
 * dE/dw the truncated label distance of each edge.  A half-step leaves its own family's chain optima
 * unchanged as functions of the inputs (the subtracted minorant vanishes on the optimal
 * labeling) but leaves that family's min-marginals tied; so the bound's derivative is the
 * one-hot of the optimal labelings of the family of the last half-step taken at the dual
 * before that half-step, and of the other family at the final dual (unique optima there
 * assumed).  Labels carry no gradient.
 *   dual          [H][W][K] the final dual of the forward call.
 *   fwd_workspace the forward's workspace, run with keep_checkpoints = 1 or 2 and the
 *                 same parameters, unchanged since.
 *   grad_cost     [H][W][K] float32 dL/dcost; grad_w_h, grad_w_v dL/dw (may be NULL).
 *   accumulate    0: outputs overwritten; 1: gradients added.
 * Per half-step (in reverse) the forward passes are recomputed from the checkpoint
 * (keep_checkpoints = 1; with 2 the forward kept what is needed), keeping every pass's
 * selection tape (see recompute_selections) or else its messages and intermediate
 * duals, then the passes are differentiated chain by chain.  The backward workspace
 * holds, with tapes, one message and one dual volume and max_pass + 1 tapes (2 tapes
 * with keep_checkpoints = 2); without, max_pass + 1 message volumes and max_pass - 1
 * dual volumes (2 and 0 with keep_checkpoints = 2); plus three adjoint volumes and
 * FP64 edge accumulators. */
size_t dm_solve_discrete_backward_workspace(dm_shape s, const dm_discrete_params* p);

int dm_solve_discrete_backward(const float* grad_minmarg, const double* grad_bounds, const void* cost,
                               dm_dtype cost_dtype, const float* w_h, const float* w_v, dm_shape s,
                               const dm_discrete_params* p, const float* dual,
                               const void* fwd_workspace, size_t fwd_workspace_bytes,
                               float* grad_cost, float* grad_w_h, float* grad_w_v, int accumulate,
                               void* workspace, size_t workspace_bytes, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Continuous refinement (paper Sec. 2.4 and Sec. 3.1).
 *
 * Minimises D(u) + sum_e w_e r((Au)_e) with (Au)_e = u_i - u_j over the grid edges and
 * r = r_{eps,delta} - r_{0, C + delta - eps*delta}  (eq. r-decompose; eps = 1, delta = 0
 * gives r(t) = min(|t|, C)), by Valkonen's non-linear primal-dual iteration
 * (eq. cont_iterates) on the reformulation with x = (u, q), y = (p, 1):
 *     u+ = prox_{tau D~}(u - tau A^T (p - q)),  q+ = prox_{tau R_-^*}(q + tau A u),
 *     p+ = prox_{sigma R_+^*}(p + sigma A (2u+ - u))     (conjugate proxes: eq. pprox).
 * The data term is replaced around u0 by the convex two-slope model D~ of Sec. 3.1 on
 * [u0 - h, u0 + h] (intersected with [0, K-1]); D between labels is the linear
 * interpolation of the cost volume along the label axis.  Slopes:
 * s_L = (D(u0) - D(u0-h))/h, s_R = (D(u0+h) - D(u0))/h, both set to their mean when
 * s_L > s_R; at the ends of the label range the missing slope copies the other.
 * Every warp re-linearises at the current u and runs n_iters iterations.  Start:
 * u = u0 = labels (as floats), p = q = 0.
 *
 * labels: [H][W] int32 in [0, K-1] (values outside are clamped).  u_out: [H][W] float32.
 * Parameter ranges: C > 0, eps in [0, 1], delta >= 0, h > 0, tau > 0, sigma > 0
 * (convergence needs tau * sigma * 8 < 1), n_warps >= 0, n_iters >= 0.
 * ------------------------------------------------------------------------------- */
typedef struct {
    float C, eps, delta, h, tau, sigma;
    int   n_warps, n_iters;
    int   keep_tape;   /* 1: the workspace also keeps, for the backward call, u0 of every warp
                          (FP64 [H][W]) and the prox branch mask of every iteration (16 bits
                          per pixel); the workspace query includes that space */
} dm_refine_params;

size_t dm_refine_continuous_workspace(dm_shape s, const dm_refine_params* p);

int dm_refine_continuous(const void* cost, dm_dtype cost_dtype, const int32_t* labels,
                         const float* w_h, const float* w_v, dm_shape s, const dm_refine_params* p,
                         float* u_out, void* workspace, size_t workspace_bytes, void* hip_stream);

/* Adjoint of dm_refine_continuous (reverse mode through the unrolled iterations; no
 * derivative in the paper - this is the exact derivative of the piecewise-linear
 * iteration map, taking at exact branch ties the branch the forward took and, for the
 * interpolated data term at an integer argument, the segment [k, k+1]).
 *   grad_u      [H][W] float32: dL/du_out.
 *   fwd_workspace: the workspace of the forward call, run with keep_tape = 1 and the
 *               same parameters, unchanged since.
 *   grad_cost   [H][W][K] float32: dL/dcost (nonzero only at the labels the data term
 *               was interpolated from).  grad_w_h / grad_w_v: dL/dw (may be NULL).
 *   accumulate  0: outputs are overwritten; 1: the gradients are added to them.
 * The labels carry no gradient (piecewise constant).  Needs its own workspace of
 * dm_refine_continuous_backward_workspace() bytes. */
size_t dm_refine_continuous_backward_workspace(dm_shape s, const dm_refine_params* p);

int dm_refine_continuous_backward(const float* grad_u, const void* cost, dm_dtype cost_dtype,
                                  const float* w_h, const float* w_v, dm_shape s,
                                  const dm_refine_params* p, const void* fwd_workspace,
                                  size_t fwd_workspace_bytes, float* grad_cost, float* grad_w_h,
                                  float* grad_w_v, int accumulate, void* workspace,
                                  size_t workspace_bytes, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Optical flow (paper Sec. 2.2 "Flow" and Sec. 3.2).  u_i in R^2: the horizontal and the
 * vertical displacement.  Labels: i in [0, K1) is the horizontal displacement i - off1,
 * j in [0, K2) the vertical displacement j - off2 (pixels).  The discretised data cost of
 * pixel (x, y) is a K2 x K1 table, stored [H][W][K2][K1]: cost[((y*W + x)*K2 + j)*K1 + i].
 * 1 <= W, H <= 16384; 1 <= K1, K2 <= 256, K1*K2 <= 4096; 0 <= off1 < K1, 0 <= off2 < K2;
 * W*H*K1*K2 < 2^32.  Errors as elsewhere (validation before any launch).
 *
 * The discrete stage decouples the two components (eq. flow decoupled costs): layer 1 has
 * the unaries f1(i) = min_j cost(i, j), layer 2 f2(j) = min_i cost(i, j), and each layer is
 * a stereo-like Dual_MM problem on the same grid and edge weights (two dm_solve_discrete
 * calls, K = K1 and K = K2).  The refinement (Sec. 3.2) runs the primal-dual iteration of
 * dm_refine_continuous on each component (the regulariser is separable over the
 * components, eq. regularizer-form) with the quadratic data model of eq. quadfit:
 * L = central first differences and Q = the positive part of the central second
 * differences (diagonal) of the bilinearly interpolated table at the current point, step
 * h, and the prox of eq. prox_flow read as
 *     u = clamp(u0 +- h, (u_hat + tau (Q u0 - L)) / (1 + tau Q))   per component,
 * the box also intersected with the label range.  u is returned in label units (the
 * displacement is u - off).
 * ------------------------------------------------------------------------------- */
typedef struct { int W, H, K1, K2, off1, off2; } dm_flow_shape;

/* Two-dimensional truncated SAD: e(x,y,i,j) = |I1(x,y) - I2(x+i-off1, y+j-off2)| (trunc if
 * the displaced position is outside I2); cost = min(trunc, mean of e over the window x.+-r,
 * y.+-r clamped to the image).  w_h / w_v (may be NULL): contrast weights of I1, as in
 * dm_build_cost_volume.  I1, I2: [H][W] float32; cost_out of out_dtype (FP16 rounded to
 * nearest even). */
int dm_build_flow_cost_volume(const float* I1, const float* I2, dm_flow_shape s, const dm_cost_params* p,
                              dm_dtype out_dtype, void* cost_out, float* w_h, float* w_v, void* hip_stream);

/* eq. flow decoupled costs: f1_out [H][W][K1], f2_out [H][W][K2], both in cost_dtype (the
 * minima are exact). */
int dm_flow_project(const void* cost, dm_dtype cost_dtype, dm_flow_shape s, void* f1_out, void* f2_out,
                    void* hip_stream);

/* Quadratic-fit refinement of both components from the two layers' labels.  p: as for
 * dm_refine_continuous (C, eps, delta, h, tau, sigma, n_warps, n_iters); keep_tape must be 0
 * (no backward: DM_ERR_UNSUPPORTED).  u1_out, u2_out: [H][W] float32 in label units.
 * State FP64 in a caller workspace of dm_refine_flow_workspace() bytes. */
size_t dm_refine_flow_workspace(dm_flow_shape s, const dm_refine_params* p);
int dm_refine_flow(const void* cost, dm_dtype cost_dtype, const int32_t* labels1, const int32_t* labels2,
                   const float* w_h, const float* w_v, dm_flow_shape s, const dm_refine_params* p,
                   float* u1_out, float* u2_out, void* workspace, size_t workspace_bytes, void* hip_stream);

/* ---------------------------------------------------------------------------------
 * Batched form: many instances of uneven size (each with its own W, H, K) solved by
 * one hipGraph launch.  dm_plan_batched picks a chain tile per labels count and chain
 * family (dm_autotune_tiles unless p fixes tile_lanes), builds the work tables and
 * captures: per half-step one persistent work-queue launch per tile class (lane
 * groups of chains pulled from an atomic counter, longest chains first; classes run
 * as parallel graph branches), the final row pass (labels), and - if rp != NULL - the
 * refinement of every instance (one launch per primal-dual iteration over all
 * instances' tiles).  The plan owns device memory (work tables, one message volume
 * per instance, refinement state) until dm_plan_destroy; the caller owns every
 * instance buffer, which must stay valid and at the same addresses.
 * dm_run_batched replays the graph on hip_stream.  Instances with warm_start = 0 get
 * dual := 0 at the start of every run.  All instances share the cost dtype and the
 * parameters.  An instance with a bounds buffer gets, per run, its lower bound (the
 * row optima of the final pass plus the column optima at the final dual, eq. DD-dual)
 * and the energy of its labels, FP64, the same quantities as dm_solve_discrete's
 * bounds_out (sums in another fixed order).  An instance with a minmarg buffer gets the
 * final row pass's normalized min-marginals (Sec. 2.3, the min-marginals of the
 * horizontal family at the final dual), bit for bit dm_solve_discrete's minmarg_out.
 * ------------------------------------------------------------------------------- */
typedef struct {
    dm_shape s;
    const void* cost;      /* [H][W][K] of the plan's cost dtype                    */
    const float* w_h;      /* [H][W-1]                                              */
    const float* w_v;      /* [H-1][W]                                              */
    int32_t* labels;       /* [H][W] output                                         */
    float* dual;           /* [H][W][K] dual state                                  */
    float* u;              /* [H][W] refined disparities (required with refinement) */
    double* bounds;        /* device [2] = {LB, E(labels)} per run, or NULL          */
    float* minmarg;        /* [H][W][K] output, 16-byte aligned, or NULL             */
} dm_instance;

int dm_plan_batched(const dm_instance* inst, int n, dm_dtype cost_dtype, const dm_discrete_params* p,
                    const dm_refine_params* rp, void** plan_out);

/* Batched forward + backward (the differentiation workload): per instance Dual_MM
 * keeping what its backward needs (p->keep_checkpoints 1 or 2), the refinement if
 * rp != NULL (its keep_tape is taken as 1), then the refinement adjoint (if grad_u is
 * given) and the Dual_MM adjoint, added into grad_cost / grad_w_h / grad_w_v - the calls
 * dm_solve_discrete, dm_refine_continuous, dm_refine_continuous_backward and
 * dm_solve_discrete_backward of this header, with their meaning, captured once into
 * one hipGraph.  With grad_cost NULL for every instance the plan is the forward only
 * (Dual_MM and the refinement; any keep_checkpoints).  The instances run on n_streams
 * (1..16) forked streams, largest (W*H*K) first to the stream with the least work so
 * far: instances advance through their half-steps independently, those of one stream
 * one after another, sharing that stream's workspaces, which the plan owns.  Outputs per run:
 * labels, dual, minmarg and bounds (each may be NULL but labels and dual), u; the
 * gradients overwritten.  Loss inputs per instance (device, read at run time):
 * grad_minmarg [H][W][K], grad_bounds [2] = {dL/dLB, dL/dE}, grad_u [H][W] (each may be
 * NULL).  The caller owns every instance buffer (same addresses for every run).
 * dm_run_batched replays the graph, dm_plan_destroy frees the plan.  Each run starts
 * from dual 0 (warm_start must be 0). */
typedef struct {
    dm_shape s;
    const void* cost;            /* [H][W][K] of the plan's cost dtype                */
    const float* w_h;            /* [H][W-1]                                          */
    const float* w_v;            /* [H-1][W]                                          */
    int32_t* labels;             /* [H][W] output                                     */
    float* dual;                 /* [H][W][K] output (the final dual)                 */
    float* minmarg;              /* [H][W][K] output or NULL                          */
    double* bounds;              /* [2] output {LB, E(labels)} or NULL                */
    float* u;                    /* [H][W] refined disparities (with refinement)      */
    const float* grad_minmarg;   /* [H][W][K] dL/dminmarg or NULL                     */
    const double* grad_bounds;   /* [2] {dL/dLB, dL/dE} or NULL                       */
    const float* grad_u;         /* [H][W] dL/du or NULL                              */
    float* grad_cost;            /* [H][W][K] float32 output (NULL: forward only)     */
    float* grad_w_h;             /* [H][W-1] output or NULL                           */
    float* grad_w_v;             /* [H-1][W] output or NULL                           */
} dm_grad_instance;

int dm_plan_batched_grad(const dm_grad_instance* inst, int n, dm_dtype cost_dtype, const dm_discrete_params* p,
                         const dm_refine_params* rp, int n_streams, void** plan_out);

int dm_run_batched(void* plan, void* hip_stream);
size_t dm_plan_device_bytes(const void* plan);
void dm_plan_destroy(void* plan);

/* ---------------------------------------------------------------------------------
 * Kernel profiler.  While enabled, every kernel launch of the library is bracketed by
 * HIP events recorded on the launch stream, and tagged with a kind and with the
 * algorithmic HBM bytes of that launch (bytes the method must move, not counters).
 * dm_profiler_query waits for the recorded events and returns, for one kind, the
 * number of launches, the summed event time and the summed algorithmic bytes.
 * Host-side state, process-wide; not thread-safe against concurrent solver calls.
 * ------------------------------------------------------------------------------- */
typedef enum {
    DM_PROF_SWEEP_H = 0,          /* horizontal half-step (rows of F)              */
    DM_PROF_SWEEP_V = 1,          /* vertical half-step (columns of G)             */
    DM_PROF_SWEEP_FINAL = 2,      /* final row min-marginal / label pass           */
    DM_PROF_SWEEP_OPT = 3,        /* column optimum pass for the bound             */
    DM_PROF_BOUNDS = 4,           /* energy / bound reductions                     */
    DM_PROF_COST_VOLUME = 5,      /* SAD cost volume + contrast weights            */
    DM_PROF_REFINE_LINEARIZE = 6, /* per-warp data-term linearisation              */
    DM_PROF_REFINE_ITER = 7,      /* primal-dual iteration                         */
    DM_PROF_OTHER = 8,            /* fills, copies                                 */
    DM_PROF_ADJOINT_H = 9,        /* adjoint of a horizontal half-step             */
    DM_PROF_ADJOINT_V = 10,       /* adjoint of a vertical half-step               */
    DM_PROF_ADJOINT_FINAL = 11,   /* adjoint of the final row pass                 */
    DM_PROF_RECORD_H = 12,        /* record-mode horizontal half-step: the forward's with
                                     keep_checkpoints = 2, or the backward's recompute   */
    DM_PROF_RECORD_V = 13,        /* record-mode vertical half-step (likewise)          */
    DM_PROF_CENSUS = 14,          /* Census + Hamming cost volume (without the weights) */
    DM_PROF_LR_CHECK = 15,        /* left-right consistency check                       */
    DM_PROF_FLOW_COST = 16,       /* two-dimensional SAD flow cost (without the weights) */
    DM_PROF_FLOW_PROJECT = 17,    /* decoupled layer costs of the flow                  */
    DM_PROF_KINDS = 18
} dm_prof_kind;

/* kind_mask != 0: clear all records and record launches of the kinds whose bit
 * (1 << kind) is set; kind_mask == 0: stop recording (records stay queryable). */
int dm_profiler_enable(unsigned kind_mask);
int dm_profiler_query(int kind, long long* launches, double* total_ms, double* alg_bytes);

/* Status text for a dm_status value, and the thread-local detail of the last error. */
const char* dm_status_string(int status);
const char* dm_last_error_message(void);

/* Library build identifier (gfx target and feature list). */
const char* dm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DMATCH_H */
