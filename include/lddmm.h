/*
 * lddmm.h -- C ABI of the masked-LDDMM registration library for AMD MI355X (gfx950).
 *
 * Method: Kutten et al., "Deformably Registering and Annotating Whole CLARITY
 * Brains to an Atlas via Masked LDDMM", Proc. SPIE 9896 (2016).
 *
 *   Methods, Registration: minimise by gradient descent
 *       E(v) = int_0^1 ||L v_t||^2 dt + sigma^-2 ||J0 o phi_10 - J1||^2,
 *       L = (-alpha Lap + gamma) I_3 ;  gamma = sigma = 1 by convention ;
 *       v discretised in time; phi_10 pulls the template into target space.
 *   Methods, Preprocessing: Mask-LDDMM replaces I0, I1 by the masks M0, M1
 *       (channel weights {1, 0}); the masked images M*I form the second channel.
 *   Methods, Postprocessing: labels are deformed with nearest-neighbour
 *       interpolation (L0 o phi^-1).
 *
 * Conventions shared by every call
 *   - All array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *     owned by the caller.  The library never allocates or frees device memory;
 *     scratch comes from the caller's workspace.
 *   - Scalar fields are contiguous FP32, index = (z*ny + y)*nx + x (x fastest).
 *     Vector fields are 3 consecutive planes (x, y, z components).  The velocity
 *     is [T][3][P] where P is the computational grid of the finest level
 *     (lddmm_comp_grid): each axis of the user grid N padded at the high end to a
 *     7-smooth length (and, with several levels, nested: P = 2^(L-1) * P_coarsest).
 *   - Displacements u = phi - id are in the physical units of `spacing`.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *     marked async only enqueue work; lddmm_register synchronises once at exit.
 *   - Errors: arguments are checked on the host before any launch; a bad
 *     argument returns LDDMM_EINVAL and enqueues nothing.  A HIP launch/runtime
 *     error returns LDDMM_EHIP.  Numeric trouble in the async calls shows up as
 *     NaN in their FP64 outputs.
 *   - Calls are reentrant across distinct workspaces; two calls that share a
 *     workspace must be ordered on one stream.
 */
#ifndef LDDMM_H
#define LDDMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LDDMM_OK          0
#define LDDMM_EINVAL     -1   /* null pointer, size < 2 or > LDDMM_MAX_DIM, T < 1,
                                 alpha/gamma/sigma/spacing <= 0, workspace too small */
#define LDDMM_EHIP       -2   /* HIP runtime or launch error */
#define LDDMM_ENONFINITE -3   /* energy not finite (NaN/Inf velocity or inputs) */
#define LDDMM_ESCRATCH   -4   /* lddmm_gradient_noalloc: the problem needs more than
                                 LDDMM_SCRATCH_BYTES of workspace */
#define LDDMM_WFOLD       1   /* warning: the returned v folds: min over j < T and the
                                 finest computational grid of det D(phi_{t_j,1}) <= 0
                                 (np.gradient stencil); result written */
#define LDDMM_WGUARD      2   /* warning: a level stopped after LDDMM_MAX_HALVINGS step halvings */

#define LDDMM_GRAD_V      0   /* Beg's gradient in V: g_j = 2 v_j - K b_j */
#define LDDMM_GRAD_L2     1   /* exact gradient dE/dv of the discrete energy */

#define LDDMM_INTERP_LINEAR  0
#define LDDMM_INTERP_NEAREST 1
#define LDDMM_F32 0
#define LDDMM_I32 1

#define LDDMM_MAX_LEVELS    4
#define LDDMM_MAX_DIM       1024
#define LDDMM_MAX_T         64
#define LDDMM_MAX_HALVINGS  10
#define LDDMM_TRACE_COLS    8   /* E, R, D, step, min det, image SSD, accepted, E_best */

/* flags */
#define LDDMM_FLAG_RECOMPUTE_PHI 1   /* exact gradient: recompute phi_t from checkpoints */
#define LDDMM_FLAG_RK4           2   /* maps by fourth-order Runge-Kutta departure points
                                        (the paper's integrator, Methods, Registration):
                                        along each step's characteristic, v_j sampled at the
                                        RK4 stages, vbar = (k1 + 2 k2 + 2 k3 + k4)/6 replaces
                                        v_j(x) in both sweeps.  Single-problem calls only
                                        (lddmm_register_batched returns LDDMM_EINVAL), and
                                        lddmm_gradient kind LDDMM_GRAD_L2 (exact reverse mode
                                        of the first-order step) returns LDDMM_EINVAL. */

/* User grid N (voxels) and the voxel spacing h of the finest level. */
typedef struct {
  int32_t nx, ny, nz;
  double spacing;
} lddmm_grid;

/* Constants of the objective (Methods, Registration) and of the descent. */
typedef struct {
  double alpha, gamma, sigma;        /* L = (-alpha Lap + gamma) I3 ; data weight 1/sigma^2 */
  int32_t n_timesteps;               /* T: v is piecewise constant on T intervals */
  int32_t n_levels;                  /* pyramid levels, each halving the resolution */
  int32_t iters[LDDMM_MAX_LEVELS];   /* iteration slots per level, coarsest first */
  double step;                       /* gradient step epsilon (reset at each level) */
  int32_t guard;                     /* 1: reject energy increases and halve the step */
  double weight[2];                  /* channel weights {mask, masked image}; {1,0} = Mask-LDDMM */
  int32_t flags;                     /* LDDMM_FLAG_* */
  int32_t checkpoint_every;          /* exact gradient with RECOMPUTE_PHI: checkpoint spacing */
} lddmm_params;

/* One registration problem.  Images are on the user grid N. */
typedef struct {
  lddmm_grid grid;
  const float *template_mask;        /* M0 [N] */
  const float *template_image;       /* M0*I0 [N] or NULL */
  const float *target_mask;          /* M1 [N] */
  const float *target_image;         /* M1*I1 [N] or NULL (NULL iff template_image is NULL) */
  float *v;                          /* [T][3][P_finest]: in = initial velocity, out = result */
  float *phi10;                      /* out: u0_T = phi_10 - id on N, [3][N]; may be NULL */
  float *phi01;                      /* out: u1_0 = phi_01 - id on N, [3][N]; may be NULL */
  double *trace;                     /* out: per level (iters+1) rows x LDDMM_TRACE_COLS; may be NULL */
  void *workspace;                   /* caller-allocated device scratch */
  size_t workspace_bytes;            /* >= lddmm_workspace_size(&grid, params) */
} lddmm_problem;

/* Bytes of device workspace one problem needs (0 if the arguments are invalid). */
size_t lddmm_workspace_size(const lddmm_grid *grid, const lddmm_params *params);

/* Computational grid of pyramid level `level` (0 = finest): out_P = {nx, ny, nz}.
   Returns LDDMM_OK or LDDMM_EINVAL. */
int lddmm_comp_grid(const lddmm_grid *grid, const lddmm_params *params, int32_t level,
                    int32_t out_P[3]);

/* Number of trace rows a registration writes: sum over levels of (iters + 1). */
int32_t lddmm_trace_rows(const lddmm_params *params);

/*
 * Register: coarse-to-fine gradient descent on E(v) (Methods, Registration).
 * Per level: images and v_init are block-averaged from the finest grid; each
 * iteration slot either takes a gradient step v - eps*g (g = 2v - K b, Beg's
 * V-gradient) or, after a rejected trial, halves eps and retries the midpoint;
 * with guard=1 a trial is accepted iff its energy does not exceed the current
 * one.  v is upsampled (cell-centred trilinear) between levels.  The guard is
 * decided on the device; the call synchronises `stream` once at exit and
 * returns LDDMM_OK, a warning or an error, in this order of precedence:
 * LDDMM_ENONFINITE (non-finite energy), LDDMM_WGUARD (a level stopped on the
 * guard), LDDMM_WFOLD (the returned v's maps phi_{t_j,1} fold; after the
 * descent, one forward and one backward sweep of the returned v at the finest
 * level take the minimum of det(I + D u1_j) over j < T and the grid).
 * With n_problems > 1 the call is lddmm_register_batched(p, n, params, NULL, stream)
 * and returns the most severe status of the batch.
 */
int lddmm_register(lddmm_problem *p, int32_t n_problems, const lddmm_params *params,
                   void *stream);

/*
 * Batched registration of n (1..32) independent problems of uneven size with one
 * set of params (same T, levels, iterations, channel weights): every stage of
 * every iteration is one kernel launch covering all problems (tiles of problem k
 * follow those of problem k-1), so the launch count does not grow with n and
 * small problems fill the GPU together.  Each problem keeps its own workspace,
 * device-side guard and trace; results equal those of n single calls.
 * status (host, n entries, may be NULL) receives each problem's status; the
 * return value is the most severe one (an error before a warning).
 */
int lddmm_register_batched(lddmm_problem *p, int32_t n, const lddmm_params *params,
                           int32_t *status, void *stream);

/*
 * Energy of p->v (Methods, Registration: the objective E(v) = int ||L v_t||^2 dt +
 * sigma^-2 ||J0 o phi_10 - J1||^2, with the Mask-LDDMM channels of Methods,
 * Preprocessing) on the single-level grid (n_levels ignored; h = grid.spacing):
 * out4 (device, 4 doubles) = {E, R, D, image SSD}, with
 *   R = dt h^3 sum_j sum_x |L v_j|^2 (periodic 7-point Laplacian),
 *   D = h^3/sigma^2 sum_c w_c sum_x (J0c o phi_10 - J1c)^2,
 *   image SSD = h^3 sum_x (M0I0 o phi_10 - M1I1)^2 (NaN without images).  Async.
 */
int lddmm_energy(const lddmm_problem *p, const lddmm_params *params, double *out4,
                 void *stream);

/*
 * Gradient of E at p->v (Methods, Registration: the gradient that the paper's
 * gradient descent follows, after Beg et al. 2005, which it cites), single
 * level: kind LDDMM_GRAD_V writes Beg's V-gradient
 *   g_j = 2 v_j - K b_j,
 *   b_j = (2/sigma^2) det(D phi_{t_j,1}) sum_c w_c (r_c o phi_{t_j,1}) grad(J0c o phi_{t_j,0}),
 * r_c = J0c o phi_10 - J1c; kind LDDMM_GRAD_L2 writes the exact derivative of
 * the discrete energy (reverse mode through the semi-Lagrangian sweep, with the
 * adjoint of trilinear sampling).  grad is [T][3][P]; out4 as lddmm_energy.  Async.
 */
int lddmm_gradient(const lddmm_problem *p, const lddmm_params *params, int32_t kind,
                   float *grad, double *out4, void *stream);

/*
 * lddmm_gradient without a caller workspace, for callers that cannot allocate
 * device memory at all (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Arguments, results and errors are those of
 * lddmm_gradient, except that p->workspace and p->workspace_bytes are ignored:
 * the scratch is a static device array of LDDMM_SCRATCH_BYTES (256 MiB) in the
 * library, one per GPU, held from the first use on that GPU until the process
 * ends.  A problem whose workspace (lddmm_workspace_size with n_levels = 1, for
 * its channel count) exceeds it returns LDDMM_ESCRATCH before any launch; 64^3
 * with T = 10 and 80^3 with T = 4 fit.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  Every call on one GPU shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU (two
 * streams, or two host threads) race and give undefined results, so order them
 * on one stream.  The first call on a GPU looks up the array's address
 * (hipGetSymbolAddress) with that GPU current.  Async.
 */
#define LDDMM_SCRATCH_BYTES (256ull << 20)
int lddmm_gradient_noalloc(const lddmm_problem *p, const lddmm_params *params, int32_t kind,
                           float *grad, double *out4, void *stream);

/*
 * Deform an image or a label map by a displacement (Methods, Postprocessing):
 *   dst(x) = src(x + u(x)/h), u [3][N] in physical units, h = grid->spacing.
 * LINEAR: trilinear, zero outside (dtype must be LDDMM_F32).
 * NEAREST: src[floor(y + 1/2)], zero outside (LDDMM_F32 or LDDMM_I32 labels); the
 * rounding is decided in FP32 from the displacement alone: index i +
 * floor(u * (1/h) + 1/2) per axis, with 1/h rounded to FP32 once, so a position
 * within FP32 rounding of a half-integer can round either way against an FP64
 * evaluation of the same formula.  Async.
 */
int lddmm_apply(const lddmm_grid *grid, const float *u, const void *src, int32_t interp,
                int32_t dtype, void *dst, void *stream);

/*
 * Apply K = (L^dagger L)^-1 (Methods, Registration) to a vector field on the
 * computational grid P = {nx, ny, nz} (each axis 7-smooth) by a 3D DFT:
 * out = IDFT((gamma + alpha lambda(k))^-2 DFT(b)), lambda the periodic 7-point
 * Laplacian symbol with spacing h.  b, out [3][P] (may alias).  Workspace from
 * lddmm_smooth_workspace_size.  Async.
 */
size_t lddmm_smooth_workspace_size(const int32_t P[3]);
int lddmm_smooth(const int32_t P[3], double spacing, double alpha, double gamma,
                 const float *b, float *out, void *workspace, size_t workspace_bytes,
                 void *stream);

/* Masks by threshold (Methods, Mask Generation): M = 1[I > tau], MI = M*I, on N. Async. */
int lddmm_make_mask(const lddmm_grid *grid, const float *image, float tau, float *mask,
                    float *masked_image, void *stream);

/* Mask application (Methods, Preprocessing): out = image where mask > 0, else 0,
 * on N (device, float32; out may alias image).  Async; LDDMM_EINVAL for a null
 * pointer or an axis outside [1, LDDMM_MAX_DIM]. */
int lddmm_mask_image(const lddmm_grid *grid, const float *image, const float *mask, float *out,
                     void *stream);

/*
 * Histogram matching of the Image-LDDMM preprocessing (Methods, Preprocessing):
 * the masked source (template) image is mapped so that its in-mask intensity
 * distribution matches that of the masked reference (target) image.
 *  - Histograms: n_bins equal-width bins over [lo, hi], the in-mask (mask > 0)
 *    minimum and maximum of each image; only in-mask voxels are counted.  The
 *    bin of x is floor((x - lo) * (n_bins / (hi - lo))) evaluated in float32,
 *    clamped to the last bin (bin 0 for a constant image).
 *  - Quantiles: the p-quantile of a histogram is where its piecewise-uniform
 *    cumulative distribution (each bin's count spread evenly over the bin)
 *    reaches p.  The match points are lo, the quantiles at p = k/(n_points+1)
 *    for k = 1..n_points, and hi, for both images (FP64).
 *  - Map: between neighbouring source points, the straight line through the
 *    matched pairs (FP64, rounded once to float32); a value at or above the
 *    last source point maps to the reference maximum.
 * out[i] = mapped src[i] where src_mask[i] > 0, else 0; all zero if either mask
 * is empty.  The paper uses n_bins = 32 and n_points = 8.
 * src, src_mask, out: [src_grid N]; ref, ref_mask: [ref_grid N]; device float32;
 * the two grids may differ; out must not alias an input.
 * points (device, may be NULL): out, [2][n_points + 2] doubles, source points
 * then reference points.  counts (device, may be NULL): out, [2][n_bins] int64
 * bin counts, source then reference.
 * workspace: device scratch of lddmm_histogram_match_workspace_size bytes
 * (caller-owned, no state kept between calls).
 * Async on `stream`.  Returns LDDMM_OK, LDDMM_EINVAL (null pointer, an axis
 * outside [1, LDDMM_MAX_DIM], n_bins outside [1, LDDMM_HIST_MAX_BINS], n_points
 * outside [0, LDDMM_HIST_MAX_POINTS], workspace too small; nothing launched) or
 * LDDMM_EHIP.
 */
/*
 * Rigid and affine pre-alignment (Methods, Registration): gradient descent on
 * the mean squared error between the template image, sampled through an affine
 * sampling map S, and the target image.
 *  - S maps target positions to template positions, x = S(y) = B y + c, in
 *    physical coordinates (voxel (i, j, k) of a grid with spacing h sits at
 *    h (i, j, k)).  S = R^-1 in the rigid stage and R^-1 A^-1 in the affine
 *    stage, so the template resampled through S is I0 o R^-1 (A^-1).
 *  - MSE(S) = (1/n1) sum over target voxels y of (I0(S(y)) - I1(y))^2, with I0
 *    trilinear in index coordinates S(y)/h0 and zero outside.  Its gradient is
 *    the exact derivative of that interpolant: G_B = (2/n1) sum r g (y - y_c)^T
 *    and G_c' = (2/n1) sum r g, with y_c the target centre and c' = B y_c + c.
 *  - A step from the current iterate uses eps for c' and eps / rho^2 for the
 *    linear part (rho^2: mean squared distance of the target voxels from y_c).
 *    Rigid: B <- B exp(-eps/rho^2 [w]_x), w_k = <G_B, B [e_k]_x> (B stays a
 *    rotation).  Affine: B <- B - eps/rho^2 G_B.
 *  - Guard: a candidate whose MSE exceeds the current iterate's is rejected
 *    and eps halved; more than max_halvings consecutive rejections stop the
 *    descent.
 */
#define LDDMM_ALIGN_RIGID  0
#define LDDMM_ALIGN_AFFINE 1
#define LDDMM_ALIGN_TRACE_COLS 28   /* MSE, step, accepted, halvings, S[12], G_B[9], G_c'[3] */
typedef struct {
  int32_t mode;             /* LDDMM_ALIGN_RIGID or LDDMM_ALIGN_AFFINE */
  int32_t iters;            /* descent slots after the starting evaluation */
  double step;              /* eps: translation step (squared length per unit MSE gradient) */
  int32_t max_halvings;     /* consecutive rejections before the descent stops */
} lddmm_align_params;

/* Bytes of device workspace lddmm_align needs for a target grid (0 if invalid). */
size_t lddmm_align_workspace_size(const lddmm_grid *target_grid);

/*
 * Run the descent.  template_image [template N], target_image [target N]: device
 * float32 (the grids may differ; each grid's spacing is its voxel size).
 * affine: device, 12 doubles, row-major [B | c]: in = starting map (the identity
 * with the grid centres lined up, or the rigid result for the affine stage),
 * out = the final iterate.  trace (device, may be NULL): rows 0..iters of
 * LDDMM_ALIGN_TRACE_COLS doubles; row 0 is the start, row s the candidate of
 * slot s (its MSE, the step it used, 1 if accepted, the consecutive
 * rejections), then the current iterate after the slot and its gradient; rows
 * after a stop are not written.  workspace: lddmm_align_workspace_size bytes,
 * caller-owned.  Async: 2 (iters + 1) + 2 launches, no host synchronisation.
 * Returns LDDMM_OK, LDDMM_EINVAL (null pointer, an axis outside [1,
 * LDDMM_MAX_DIM], spacing not positive, bad mode, iters or max_halvings < 0,
 * step not positive, workspace too small; nothing launched) or LDDMM_EHIP.
 */
int lddmm_align(const lddmm_grid *template_grid, const float *template_image,
                const lddmm_grid *target_grid, const float *target_image,
                const lddmm_align_params *params, double *affine, double *trace,
                void *workspace, size_t workspace_bytes, void *stream);

/*
 * Resample through an affine map composed with a displacement (Methods,
 * Registration: phi^-1 = R^-1 A^-1 phi_10):
 * dst(y) = src(S(y + u(y))) on dst_grid, S = affine (device, 12 doubles [B | c]),
 * u = displacement in physical units on dst_grid ([3][N], device; NULL: none),
 * src on src_grid.  LINEAR: trilinear, zero outside (LDDMM_F32).  NEAREST:
 * src at floor(x/h + 1/2), zero outside (LDDMM_F32 or LDDMM_I32 labels).
 * With u = phi_10 - id from lddmm_register this is the label transfer
 * L0 o phi^-1; with u = NULL it resamples the template onto the target grid
 * (J0 = I0 o R^-1 A^-1).  Async; LDDMM_EINVAL for invalid arguments.
 */
int lddmm_apply_affine(const lddmm_grid *dst_grid, const float *u, const double *affine,
                       const lddmm_grid *src_grid, const void *src, int32_t interp,
                       int32_t dtype, void *dst, void *stream);

#define LDDMM_HIST_MAX_BINS   1024
#define LDDMM_HIST_MAX_POINTS 62
size_t lddmm_histogram_match_workspace_size(const lddmm_grid *src_grid,
                                            const lddmm_grid *ref_grid, int32_t n_bins);
int lddmm_histogram_match(const lddmm_grid *src_grid, const float *src, const float *src_mask,
                          const lddmm_grid *ref_grid, const float *ref, const float *ref_mask,
                          int32_t n_bins, int32_t n_points, float *out, double *points,
                          int64_t *counts, void *workspace, size_t workspace_bytes,
                          void *stream);

/*
 * Kernel-class timing with HIP events recorded on the launch stream around each
 * launch of the selected classes (bit k of class_mask = class k below) whose
 * grid has at least min_voxels voxels.
 * lddmm_profile_begin clears the record and starts recording for every later
 * call of this process; lddmm_profile_end synchronises the recorded events,
 * writes per class the summed duration (ms), the number of launches and the
 * number of grid voxels those launches covered (arrays of LDDMM_PROF_CLASSES,
 * host memory, may be NULL) and stops recording.  Not thread-safe.
 */
#define LDDMM_PROF_FORWARD   0   /* forward map step + template warp + energy partials,
                                    interior steps 0 < j < T-1 */
#define LDDMM_PROF_BACKWARD  1   /* backward map step + Jacobian + body force, the steps
                                    that compute both a map and a body force */
#define LDDMM_PROF_FFT_X     2   /* x forward pass of K (real -> half spectrum) */
#define LDDMM_PROF_FFT_Y     3   /* y forward pass */
#define LDDMM_PROF_FFT_ZK    4   /* z pass: forward, K_hat, inverse */
#define LDDMM_PROF_FFT_YINV  5   /* y inverse pass */
#define LDDMM_PROF_FFT_XINV  6   /* x inverse pass + velocity update */
#define LDDMM_PROF_OTHER     7   /* retry, guard decision, pyramid, setup */
#define LDDMM_PROF_HIST_RANGE  8 /* histogram matching: in-mask range (two launches) */
#define LDDMM_PROF_HIST_COUNT  9 /* histogram matching: bin counts, totals, point table (three launches) */
#define LDDMM_PROF_HIST_APPLY 10 /* histogram matching: intensity map */
#define LDDMM_PROF_ALIGN     11  /* pre-alignment: MSE and gradient pass */
#define LDDMM_PROF_FORWARD_EDGE  12  /* forward steps j = 0 and j = T-1 (the last also
                                        forms the residual and the data terms) */
#define LDDMM_PROF_BACKWARD_EDGE 13  /* backward steps with a map but no body force
                                        (the first) or a body force but no map (the last) */
#define LDDMM_PROF_CLASSES   14
int lddmm_profile_begin(uint32_t class_mask, int64_t min_voxels);
int lddmm_profile_end(double *ms_total, int64_t *launches, int64_t *voxels);

/*
 * Launch-shape tunables (process-wide; results are identical for every value,
 * only speed changes).  LDDMM_TUNE_SWEEP_BLOCKS: blocks of the forward and
 * backward sweep kernels (rounded to a multiple of 8, clamped to [8, 4096];
 * default 4096).  LDDMM_TUNE_FFT_X_ELEMS: complex values one block of the x
 * passes of K holds in LDS (row pairs per block = value / (3 nx), 1..8; clamped
 * to [256, 8192]; default 2048).  LDDMM_TUNE_FFT_COLS / LDDMM_TUNE_FFT_ZCOLS:
 * kx columns per tile of the y / the z pass (rounded down to a power of two in
 * [2, 32], then halved while columns x length exceeds 4096; defaults 16 and 8).
 * LDDMM_TUNE_STAGED_MIN_BLOCKS: the backward sweep uses its LDS-staged kernel
 * on grids that give at least this many blocks (one per 64 x 4 column and
 * z-slab; default 2048, at most 4096 blocks).  LDDMM_TUNE_FWD_TILES: the
 * forward sweep gives each thread a column of one xy plane block (256 voxels)
 * and a run of consecutive z-planes, with at most this many blocks where that
 * allows one run per plane block (whole runs, rounded up to a multiple of 8, at
 * most 4096; default 1792), on grids whose xy plane needs
 * at most 4089 such blocks; 0 selects the grid-stride forward sweep with
 * LDDMM_TUNE_SWEEP_BLOCKS blocks on every grid.  Block counts and traversals
 * change only the order of the FP64 energy partial sums.  A value applies to
 * calls enqueued after it is set.  Returns LDDMM_OK or LDDMM_EINVAL (unknown
 * `which`, or value < 1; value < 0 for LDDMM_TUNE_FWD_TILES and
 * LDDMM_TUNE_FFT_FUSED_LDS).
 */
#define LDDMM_TUNE_SWEEP_BLOCKS 0
#define LDDMM_TUNE_FFT_X_ELEMS  1
#define LDDMM_TUNE_FFT_COLS     2
#define LDDMM_TUNE_FFT_ZCOLS    3
#define LDDMM_TUNE_STAGED_MIN_BLOCKS 4
#define LDDMM_TUNE_FWD_TILES    5
#define LDDMM_TUNE_FWD_STAGED_MIN_BLOCKS 6   /* the forward sweep reads its map gather
                                        from an LDS-staged ring of u0 planes (64 x 4
                                        columns marching z-slabs, as the staged backward)
                                        on grids that give at least this many blocks
                                        (at most 4096 blocks); it takes precedence over
                                        LDDMM_TUNE_FWD_TILES there.  Default 2048. */
#define LDDMM_TUNE_FFT_FUSED_LDS 7  /* K transforms x and y in one pass each way,
                                        with one component's xy plane of the half
                                        spectrum in LDS, on grids whose (nx, ny) has a
                                        fused plan ((140, 80), (70, 40), (32, 32),
                                        (64, 64)) and whose plane needs at most this
                                        many bytes of LDS; 0 never fuses.  Default
                                        81920.  The fused passes pack rows of one
                                        component where the separate passes pack
                                        rows across components, so K b differs in
                                        rounding only (FP32). */
#define LDDMM_TUNE_K_TIME_BATCH 8   /* 1 (default): on the levels of lddmm_register
                                        with at most 2^21 voxels, the backward sweep
                                        keeps the T body forces and then applies K
                                        and the update to all of them, one launch
                                        per pass; 0: K and the update after each
                                        step.  Same results; the workspace holds the
                                        buffers either way.  Values other than 0
                                        and 1: LDDMM_EINVAL. */
int lddmm_set_tunable(int32_t which, int32_t value);

/* Device copy of n floats, src -> dst (device, not overlapping): the library's
 * copy kernel, the one that moves v between pyramid levels; with a large n it is
 * also a probe of the attainable memory bandwidth.  Async; LDDMM_EINVAL for a
 * null pointer with n > 0 or n < 0. */
int lddmm_copy(const float *src, float *dst, int64_t n, void *stream);

/* Human-readable text of a status code (static storage). */
const char *lddmm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LDDMM_H */
