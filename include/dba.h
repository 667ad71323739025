/*
 * dba.h -- C ABI of the MI355X ADMM bundle-adjustment library (libdba.so).
 *
 * The library runs the data-parallel hot path of distributed bundle
 * adjustment by ADMM (Ramamurthy et al., "Distributed Bundle Adjustment",
 * Sec. 3.1): every observation z_ij owns a local copy (y_j^i, x_i^j) of its
 * camera and point; one iteration solves each copy's local problem (Eq. 9),
 * averages copies plus scaled duals into consensus values (Eqs. 10, 11),
 * updates the scaled duals (Eqs. 12, 13), and evaluates primal/dual residual
 * norms (with optional residual balancing of rho).
 *
 * Conventions for every call:
 *   - All pointer arguments are HOST memory owned by the caller.  Inputs are
 *     copied before the call returns; outputs are written before it returns.
 *   - Camera vectors have 9 doubles: (w_x, w_y, w_z, t_x, t_y, t_z, f, k1, k2)
 *     -- angle-axis rotation world->camera, translation, focal length in
 *     pixels, two radial distortion terms; pixel = f (1 + k1 r^2 + k2 r^4) *
 *     (P_1/P_3, P_2/P_3) with P = R(w) X + t (Sec. 2.1, Eq. 1, extended by
 *     f, k1, k2).  Points have 3 doubles.  Observations are (camera, point,
 *     u, v) in any order; arrays are indexed by observation k = 0..n_obs-1.
 *   - Every function returns a dba_status; on error the handle state is
 *     unchanged and dba_last_error() describes the failure.
 *   - Work is enqueued on the handle's stream; calls that return data
 *     synchronise that stream.  A handle is not thread-safe.
 */
#ifndef DBA_H
#define DBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dba_handle dba_handle;

typedef enum {
    DBA_OK = 0,
    DBA_E_INVALID_ARG = -1,   /* null pointer, bad size or option */
    DBA_E_INDEX_RANGE = -2,   /* camera/point index outside [0, n) */
    DBA_E_UNOBSERVED = -3,    /* a camera or point has no observation */
    DBA_E_NONFINITE = -4,     /* non-finite input, or the iteration produced one */
    DBA_E_BEHIND_CAMERA = -5, /* an observation has depth <= 1e-6 at the initial estimate */
    DBA_E_DEVICE = -6,        /* HIP runtime error */
    DBA_E_STATE = -7          /* call not valid in the current state (e.g. no problem set) */
} dba_status;

typedef enum {
    DBA_LOSS_L2 = 0,          /* phi(s) = s */
    DBA_LOSS_HUBER = 1,       /* phi(s) = s if s <= d^2 else 2 d sqrt(s) - d^2, d = loss_param (px) */
    DBA_LOSS_STUDENT_T = 2    /* phi(s) = nu log(1 + s/nu), nu = loss_param */
} dba_loss;

typedef enum {
    DBA_PREC_FP64 = 0,        /* everything in FP64 */
    DBA_PREC_FP32_LOCAL = 1   /* local solves in FP32; consensus, duals, norms in FP64 */
} dba_precision;

typedef enum {
    DBA_START_PLAIN = 0,      /* local LM starts from the previous local copy */
    DBA_START_LEARNED = 1     /* start from the better of the copy and copy + MLP prediction */
} dba_start;

typedef enum {
    DBA_CAMERA_ANGLE_AXIS = 0, /* 9 parameters, all optimised: angle-axis w (3), t (3), focal f,
                                  radial k1, k2; pixels f (1 + k1 r^2 + k2 r^4) (P1/P3, P2/P3) */
    DBA_CAMERA_EULER = 1       /* the camera of Sec. 2.1, Eq. (1): Euler angles (alpha, beta, gamma)
                                  and t optimised (6 parameters), R = R3(gamma) R2(beta) R1(alpha)
                                  (rotations about x, y, z), pixels f (P1/P3, P2/P3) with the known
                                  focal length f; a camera row is (alpha, beta, gamma, t, f, 0, 0) */
} dba_camera;

typedef enum {
    DBA_SOLVER_LM = 0,           /* robust Levenberg-Marquardt (lm_steps, lm_lambda0) */
    DBA_SOLVER_GAUSS_NEWTON = 1, /* the paper's solver for the l2 misfit (Sec. 3.1): the same steps
                                    without damping, every step with a finite trial taken;
                                    per-observation local solves, plain start only */
    DBA_SOLVER_LBFGS = 2         /* the paper's solver for the Huber misfit (Sec. 3.1; Nocedal &
                                    Wright, Alg. 7.4-7.5): lm_steps iterations, initial matrix
                                    diag(P + 2 w J^T J)^-1 at the iterate, at most 4 curvature pairs
                                    (kept if s.y > 1e-8 s^T P s), Armijo backtracking from step 1
                                    by halves, at most 10 trials; the solve ends when no trial is
                                    taken or the predicted decrease is below F's rounding
                                    resolution; per-observation local solves, plain start only */
} dba_local_solver;

typedef struct dba_options {
    int32_t device;           /* HIP device ordinal */
    void *stream;             /* hipStream_t to enqueue on; NULL: a stream the handle creates */
    int32_t precision;        /* dba_precision */
    int32_t loss;             /* dba_loss (phi_m of Eq. 8) */
    double loss_param;        /* Huber delta in pixels, or Student-t nu */
    double rho_x, rho_y;      /* penalty weights of Eq. (8), points and cameras (> 0) */
    int32_t rho_balancing;    /* 1: residual balancing of rho after every iteration */
    double rb_mu, rb_tau;     /* balancing: act when one residual exceeds mu x the other; scale by tau */
    double rho_min, rho_max;  /* balancing clamps */
    int32_t lm_steps;         /* local-solver steps per local solve (LM: counting rejected ones;
                                 L-BFGS: iterations) (1..64) */
    double lm_lambda0;        /* initial Marquardt damping of each local solve */
    int32_t start;            /* dba_start */
    int32_t learned_lm_steps; /* LM steps after the learned start (1..64) */
    int32_t use_graph;        /* 1: replay iterations from a captured hipGraph */
    int32_t block_waves;      /* local-solve workgroup size in wavefronts (1,2,4,8); 0: autotune */
    int32_t persistent;       /* local solve: 1 persistent grid, 0 one workgroup per tile, -1 autotune */
    int32_t camera_blocks;    /* 0: one local problem per observation (Eqs. 9-13);
                                 1: generalised local updates (Sec. 3.1.4, Eqs. 14-15): the
                                 observations of a camera, in ascending point order, form blocks
                                 of up to 64 that share one camera copy; each block's problem
                                 (9 + 3 x observations unknowns) is one local solve; not with the
                                 learned start */
    int32_t block_points;     /* with camera_blocks: observations (points) per block, the pi of
                                 Sec. 3.1.4, 1..64; 0 means 64.  Must be 0 without camera_blocks */
    int32_t camera_model;     /* dba_camera; the Euler camera not with the learned start */
    int32_t local_solver;     /* dba_local_solver */
    int32_t block_cameras;    /* with camera_blocks: cameras per block, the kappa of Sec. 3.1.4:
                                 1 (the blocks above) or 2: cameras in consecutive pairs, each
                                 pair's observed points in ascending order in runs of
                                 block_points (0: 64); a block holds one run with ONE copy of each
                                 of its points and of each pair camera that observes them, and its
                                 local problem couples them (18 + 3 x points unknowns, Schur
                                 complement on the points, an 18x18 camera system).  Must be 1
                                 without camera_blocks */
    int32_t segment_schedule; /* point-consensus segment schedule: 1 a thread per point sums its
                                 records; 2 a thread per group of up to 8 consecutive records
                                 (more for tracks over 512), the point's group sums then added
                                 in order; 3 as 2 with each wave's records staged through LDS
                                 by coalesced loads.  All sum each point's records in the same
                                 groups and order, so the results are bitwise identical; 0:
                                 autotune */
} dba_options;

/* Fills *opt with the defaults: device 0, NULL stream, FP64, Huber 2 px,
 * rho 1, no balancing (mu 10, tau 2, clamps 1e-6..1e6), 5 LM steps,
 * lambda0 1e-3, plain start, 2 learned steps, graphs on, autotune (local and
 * segment schedules), one
 * local problem per observation (camera_blocks 0, block_points 0), the
 * 9-parameter angle-axis camera, robust LM. */
int dba_default_options(dba_options *opt);

/* Creates a handle on opt->device.  *out receives the handle. */
int dba_create(const dba_options *opt, dba_handle **out);

/* Frees the handle and all device memory it owns.  NULL is allowed. */
void dba_destroy(dba_handle *h);

/* Message of the last failed call on this handle ("" if none).  The string
 * stays valid until the next call on the handle. */
const char *dba_last_error(const dba_handle *h);

/* One bundle-adjustment problem (the statement of Sec. 2.2): n_cams
 * cameras y_j, n_points points x_i, and n_obs observations z_ij, i in S(j). */
typedef struct dba_problem_desc {
    int32_t n_cams, n_points;
    int64_t n_obs;
    const int32_t *obs_cam;   /* [n_obs] camera index j of observation k */
    const int32_t *obs_point; /* [n_obs] point index i of observation k */
    const double *obs_uv;     /* [2*n_obs] pixel (u, v) of observation k */
    const double *cams;       /* [9*n_cams] initial consensus cameras, rows as the options'
                                 camera_model lays them out */
    const double *points;     /* [3*n_points] initial consensus points */
} dba_problem_desc;

/* Sets one problem (equivalent to dba_set_problems with one entry).
 * Initial local copies = initial consensus, scaled duals = 0, rho from the
 * options, iteration counter 0.  Validation: indices in range
 * (DBA_E_INDEX_RANGE), all values finite (DBA_E_NONFINITE), every camera and
 * point observed at least once, since Eqs. (10)-(11) divide by the count
 * (DBA_E_UNOBSERVED), depth > 1e-6 for every observation at the initial
 * estimate (DBA_E_BEHIND_CAMERA); with the Euler camera, f > 0 and zeros in
 * slots 7, 8 of every camera row (DBA_E_INVALID_ARG). */
int dba_set_problem(dba_handle *h, int32_t n_cams, int32_t n_points, int64_t n_obs,
                    const int32_t *obs_cam, const int32_t *obs_point, const double *obs_uv,
                    const double *cams, const double *points);

/* Sets n_problems independent problems that then iterate together in the
 * same launches; each keeps its own rho, residuals and iteration count, and
 * its results are bitwise identical to running it alone. */
int dba_set_problems(dba_handle *h, int32_t n_problems, const dba_problem_desc *probs);

/* Runs n_iters ADMM iterations (Eqs. 9-13 + residual norms + optional rho
 * balancing) on every problem.  Asynchronous: returns after enqueueing.
 * n_iters >= 0. */
int dba_iterate(dba_handle *h, int32_t n_iters);

typedef struct dba_residual_report {
    double primal;            /* sqrt(sum_k |copy_k - consensus|^2) of the last iteration */
    double dual;              /* sqrt(rho_x^2 sum_i N_i |dx_i|^2 + rho_y^2 sum_j M_j |dy_j|^2) */
    double rho_x, rho_y;      /* rho used by the last iteration */
    double next_rho_x, next_rho_y; /* rho the next iteration will use */
    double rmse;              /* sqrt(sum |e|^2 / L) at the consensus estimate (want_rmse) */
    double rmse_masked;       /* same over the observations of the evaluation mask */
    double robust_cost;       /* sum phi(|e|^2) at the consensus estimate */
    double mean_error;        /* mean |e| */
    int64_t iteration;        /* iterations run so far */
    int32_t nonfinite;        /* 1 if a non-finite value was seen in the consensus */
    int32_t reserved;
} dba_residual_report;

/* Residual report of problem `problem`.  want_rmse != 0 also evaluates the
 * reprojection statistics at the current consensus (one extra pass). */
int dba_residuals(dba_handle *h, int32_t problem, int32_t want_rmse, dba_residual_report *out);

/* Marks which observations of `problem` count for rmse_masked (mask[k] != 0);
 * NULL resets to all observations. */
int dba_set_eval_mask(dba_handle *h, int32_t problem, const uint8_t *mask);

/* Consensus estimate of `problem`: cams [9*n_cams], points [3*n_points], FP64. */
int dba_get_params(dba_handle *h, int32_t problem, double *cams, double *points);

/* Full ADMM state of `problem` in the caller's observation order: local
 * copies [12*n_obs] as (y_j^i (9), x_i^j (3)) and scaled duals [12*n_obs],
 * FP64.  With camera_blocks every observation reports the camera copy and
 * dual of its block.  Either pointer may be NULL. */
int dba_get_state(dba_handle *h, int32_t problem, double *copies, double *duals);

/* Number of problems set, and the sizes of one. */
int dba_problem_info(const dba_handle *h, int32_t problem, int32_t *n_cams, int32_t *n_points,
                     int64_t *n_obs);

/* Kernel timing: while enabled, dba_iterate records HIP events around each
 * kernel on the handle's stream -- with use_graph, as event-record nodes of
 * graphs captured for timing (two per graph size, so one replay's times are
 * read while the next runs; eager launches if the capture is refused),
 * otherwise around eager launches.  Kernel ids:
 * 0 local solve, 1 consensus, 2 residual norms, 3 learned warm start.
 * enable: 0 off, 1 every kernel, 2 the local solve only (ids 0 and 3; two
 * events per iteration instead of six), 3 the local solve of the first
 * iteration of each batch of 16 (and of each single iteration after the
 * last whole batch): with use_graph that launch runs between two events
 * recorded on the stream and the rest of the batch is replayed from a graph,
 * so the timing barely slows the iterations it samples and needs no
 * event-record node inside a graph (without use_graph, every local launch);
 * other values DBA_E_INVALID_ARG.
 * dba_kernel_times returns, per id, total milliseconds and launch counts
 * since timing was enabled (synchronises the stream). */
int dba_set_kernel_timing(dba_handle *h, int32_t enable);
int dba_kernel_times(dba_handle *h, double *total_ms /*[4]*/, int64_t *launches /*[4]*/);

/* Launch schedule in use: waves per local-solve workgroup, persistent flag,
 * and number of candidate schedules the autotuner timed (0 if fixed). */
int dba_schedule(const dba_handle *h, int32_t *block_waves, int32_t *persistent, int32_t *tuned);
/* Segment schedule of the consensus in use (segment_schedule of
 * dba_options) and the number of candidates the autotuner timed (0 if
 * fixed).  Every candidate gives bitwise-identical results, so tuning on the
 * first iterations does not change them. */
int dba_segment_schedule(const dba_handle *h, int32_t *segment_schedule, int32_t *tuned);

/* ---------------------------------------------------------------------------
 * Learned warm start.  Before each local solve a small network predicts the
 * solve's update from 26 features of the observation's local problem:
 * residual at the start point (2), camera copy minus consensus (9), point
 * copy minus consensus (3), scaled duals (9 + 3).  Network 26 -> 128 -> GELU
 * -> 128 -> GELU -> 12, bf16 weights and activations, FP32 accumulation
 * (gfx950 matrix cores).  The solve starts from the better (lower F of
 * Eq. 9) of the copy and copy + prediction, ties keep the copy, and then runs
 * `learned_lm_steps` plain LM steps.  FP32 local solves only.
 * Parameter block (DBA_MLP_PARAMS floats): W1 [32][128] (rows 26..31 zero),
 * b1 [128], W2 [128][128], b2 [128], W3 [128][16] (columns 12..15 zero),
 * b3 [16]; layer l computes h W_l + b_l.  Normalisation (DBA_MLP_NORM floats):
 * feature mean [26], feature std [26], output mean [12], output std [12];
 * the network sees (f - mean) / std and predicts (delta - mean) / std.
 * ------------------------------------------------------------------------- */
#define DBA_MLP_PARAMS 22800
#define DBA_MLP_NORM 76

/* Sets the network (copied; bf16 copies made on the device). */
int dba_set_mlp(dba_handle *h, const float *params, const float *norm);
/* Reads the network's FP32 parameters and normalisation (either may be NULL). */
int dba_get_mlp(dba_handle *h, float *params, float *norm);
/* Switches the start of the local solves (dba_start) and the LM steps that
 * follow a learned start; DBA_E_STATE at the next dba_iterate if learned and
 * no network is set. */
int dba_set_start(dba_handle *h, int32_t start, int32_t learned_lm_steps);
/* Network evaluation: features [n][26] -> predicted updates [n][12]. */
int dba_mlp_forward(dba_handle *h, const float *features, int64_t n, float *delta);
/* Allocation-free network evaluation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the computation of dba_mlp_forward, with
 * DEVICE buffers owned by the caller -- features [n][26] FP32 in, predicted
 * updates [n][12] FP32 out -- enqueued on the handle's stream without a
 * synchronisation (the result is ready when the stream reaches it).  Its
 * intermediate values live in one fixed scratch array of the library per GPU
 * (DBA_NOALLOC_SCRATCH_BYTES, held until the process ends), so n is at most
 * DBA_NOALLOC_MAX_ROWS (DBA_E_INVALID_ARG beyond, DBA_E_STATE without a
 * network).  Calls that overlap on one GPU (other handles, streams or
 * threads) race on that array.  Allocates nothing: no hipMalloc, hipFree or
 * allocating library routine. */
#define DBA_NOALLOC_MAX_ROWS 65536
#define DBA_NOALLOC_SCRATCH_BYTES (DBA_NOALLOC_MAX_ROWS * 128)
int dba_mlp_forward_noalloc(dba_handle *h, const float *features, int64_t n, float *delta);
/* Mean squared error over n x 12 of the network on standardized inputs
 * x_std [n][32] (rounded to bf16 on the device) against standardized targets
 * t_std [n][16] (columns 12..15 ignored), its gradient with respect to the
 * parameter block (grad [DBA_MLP_PARAMS], may be NULL) and the outputs
 * y_out [n][16] (may be NULL).  n a multiple of 64, at most 65536. */
int dba_mlp_loss_grad(dba_handle *h, const float *x_std, const float *t_std, int32_t n, float *loss, float *grad,
                      float *y_out);
/* Runs n_iters plain ADMM iterations of the problem set; before each one
 * samples per_iter observations (seeded) and records, for each, its 26
 * features and the update of an LM run of conv_steps steps from the copy on
 * the same local problem: features [n_iters*per_iter][26], deltas [..][12].
 * FP32 local solves of one observation each only (DBA_E_INVALID_ARG with
 * camera_blocks). */
int dba_collect_pairs(dba_handle *h, int32_t n_iters, int32_t per_iter, uint64_t seed, int32_t conv_steps,
                      float *features, float *deltas);
/* Trains the network on n pairs: standardisation from the pairs, N(0,
 * 1/fan_in) initialisation (seeded), Adam (0.9, 0.999, 1e-8) with a cosine
 * learning-rate schedule from lr, mean squared error on standardized
 * targets, shuffled full batches of `batch` (a multiple of 64).  epoch_loss
 * [epochs] receives the mean training loss of each epoch (may be NULL).  The
 * trained network becomes the handle's network. */
int dba_mlp_train(dba_handle *h, const float *features, const float *deltas, int64_t n, int32_t epochs, int32_t batch,
                  double lr, uint64_t seed, float *epoch_loss);
/* One Adam step (Kingma & Ba 2015: beta 0.9, 0.999, eps 1e-8, bias
 * correction by the handle's step count) of the network's FP32 parameters
 * with a gradient computed elsewhere, grad [DBA_MLP_PARAMS] (for example a
 * sum of dba_mlp_loss_grad results over several batches or handles); the
 * padding entries of the parameter block stay zero.  dba_set_mlp and
 * dba_mlp_train start the optimiser state from zero; dba_mlp_train's steps
 * use the same update.  DBA_E_STATE without a network, DBA_E_NONFINITE for a
 * non-finite gradient entry. */
int dba_mlp_apply_gradient(dba_handle *h, const float *grad, double lr);
/* Reads the Adam state: first and second moments m, v [DBA_MLP_PARAMS]
 * (either may be NULL) and the number of steps taken since it was zeroed. */
int dba_mlp_adam_state(dba_handle *h, float *m, float *v, int64_t *step);

#ifdef __cplusplus
}
#endif
#endif
