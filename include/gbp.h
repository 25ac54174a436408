/*
 * gbp.h - C ABI of the MI355X (gfx950) Gaussian Belief Propagation
 * bundle-adjustment library.
 *
 * The library runs synchronous GBP sweeps (Ortiz et al., "Bundle Adjustment
 * on a Graph Processor", Section 5) over a keyframe / landmark /
 * reprojection-factor graph (Section 4) on one GPU. Every entry point returns
 * a gbp_status; nothing throws across the ABI. Host pointers are plain
 * row-major arrays owned by the caller; the library copies what it needs.
 * All device work is ordered on the stream given in gbp_options; calls that
 * return host results synchronise that stream.
 *
 * Conventions (shared with the paper's problem statement, Section 4):
 *   - keyframe pose x = (omega, t) in R^6, world -> camera: a world point l
 *     maps to R(omega) l + t, R(omega) = Exp(omega) (axis-angle);
 *   - landmark l in R^3, world frame;
 *   - measurement z in pixels, h(x, l) = pi(R l + t) with a pinhole
 *     projection (fx, fy, cx, cy), noise Sigma_M = sigma^2 I;
 *   - Huber threshold huber_k in pixels (Section 6; N_sigma = huber_k/sigma),
 *     huber_k <= 0 disables the robust kernel.
 */
#ifndef GBP_H
#define GBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GBP_OK = 0,
    GBP_EINVAL = -1,   /* bad argument: sizes, indices, options          */
    GBP_ENOMEM = -2,   /* device or host allocation failed / no capacity */
    GBP_EDEVICE = -3,  /* a HIP runtime call failed                       */
    GBP_ENUMERIC = -4, /* a belief was not positive definite / not finite */
    GBP_ESTATE = -5    /* call not valid in the problem's current state   */
} gbp_status;

/* Storage precision of per-factor state and messages, and of the stored
 * reference pixels of gbp_set_reference (passed in FP64; in FP32 their
 * rounding is below 1e-4 px for pixels under 2048). Measurements are kept
 * in FP64. Beliefs (covariance and mean offsets), belief sums and the
 * 6x6 / 3x3 solves are FP64 in both modes; the per-factor 2x2
 * marginalisation arithmetic is FP64 as well. */
enum { GBP_FP64 = 0, GBP_FP32 = 1 };

/* Message damping (Section 5, last paragraph): the paper damps the eta
 * message; GBP_DAMP_ETA_LAMBDA damps the Lambda message with the same
 * factor as well. */
enum { GBP_DAMP_ETA = 0, GBP_DAMP_ETA_LAMBDA = 1 };

typedef struct gbp_problem gbp_problem; /* opaque, owned by the library */

/* Variables, factors and initial estimate of one problem (Section 4). */
typedef struct {
    int32_t n_keyframes, n_landmarks, n_factors;
    const int32_t *factor_kf;      /* [n_factors] keyframe of each factor  */
    const int32_t *factor_lm;      /* [n_factors] landmark of each factor  */
    const double *kf_init;         /* [n_keyframes][6] initial (omega, t)  */
    const double *lm_init;         /* [n_landmarks][3] initial position    */
    const double *kf_anchor_info;  /* [n_keyframes] or NULL: a value a > 0
                                      replaces that keyframe's automatic
                                      prior by a*I at its initial pose      */
} gbp_graph;

typedef struct {
    double fx, fy, cx, cy; /* pinhole intrinsics, pixels            */
    double sigma_px;       /* measurement noise standard deviation  */
} gbp_camera;

typedef struct {
    const double *z;       /* [n_factors][2] measured pixels        */
} gbp_measurements;

/* Hyperparameters; gbp_default_options fills in the paper's (Section 8). */
typedef struct {
    int32_t precision;             /* GBP_FP64 | GBP_FP32                   */
    int32_t damp_mode;             /* GBP_DAMP_ETA | GBP_DAMP_ETA_LAMBDA     */
    double beta;                   /* relinearisation distance, 0.01        */
    int32_t relin_min_interval;    /* factor updates between relins, 10     */
    int32_t undamped_after_relin;  /* undamped updates after relin, 8 (>=1) */
    int32_t anneal;                /* 1: priors weaken over anneal_iters    */
    int32_t prior_anneal_iters;    /* 10 (<= 64)                            */
    double prior_weaken;           /* final prior scale, 0.01               */
    double huber_k;                /* initial Huber threshold (px), 2       */
    double zmin;                   /* minimum valid camera depth, 1e-3      */
    int32_t max_keyframes;         /* capacity for gbp_add_keyframe growth  */
    int32_t max_landmarks;         /*   (0: the created sizes)              */
    int32_t max_factors;
    void *workspace;               /* optional device memory (e.g. torch);
                                      NULL: the library allocates           */
    size_t workspace_bytes;
    void *stream;                  /* hipStream_t; NULL: default stream     */
} gbp_options;

/* Reprojection statistics at the current belief means (Section 9.1: the
 * average reprojection error; Section 9.4: a measurement is classed an
 * outlier when it lies in the linear Huber regime). */
typedef struct {
    double are_all;        /* mean |z - h(mu)| over valid factors (px)     */
    double are_quadratic;  /* mean over factors with |z - h| <= huber_k    */
    double are_ref;        /* mean |z_ref - h(mu)| over the reference mask */
    int64_t n_valid;       /* factors with camera depth > zmin             */
    int64_t n_quadratic;
    int64_t n_linear;      /* factors in the linear (outlier) regime       */
    int64_t n_invalid;     /* factors with camera depth <= zmin            */
    int64_t n_ref;         /* valid factors inside the reference mask      */
    int64_t n_linear_ref;  /* of those, in the linear regime: with the mask
                              marking true inliers, the outlier classes that
                              are false positives (Section 9.4, Fig. 7a)  */
} gbp_reproj;

/* Fill opt with the paper's hyperparameters and FP32 storage. */
void gbp_default_options(gbp_options *opt);

/* Device bytes the library needs for n problems under opt (capacity
 * included). Pass a workspace of at least this size, or NULL. */
gbp_status gbp_workspace_bytes(int32_t n_problems, const gbp_graph *graphs,
                               const gbp_options *opt, size_t *bytes);

/* Build one problem (Section 4): validates indices, orders landmarks by
 * their first observing keyframe and factors keyframe-major (within a
 * keyframe by landmark), builds a landmark CSR over the factors, copies
 * inputs to the device,
 * linearises every factor at the initial estimate, builds the automatic
 * priors and sets each belief to its prior (iteration clock t = 0).
 * Returns GBP_EINVAL for out-of-range indices or sizes. */
gbp_status gbp_create(const gbp_graph *graph, const gbp_camera *camera,
                      const gbp_measurements *meas, const gbp_options *opt,
                      gbp_problem **out);

/* Build n independent problems that run as one block-diagonal graph and
 * one launch sequence (arrays of n graphs / cameras / measurements). */

/* Largest batch: the keyframes, the landmarks and the factors of all of a
 * batch's problems (growth capacities included) may each number at most
 * this; gbp_create, gbp_create_batch and gbp_workspace_bytes return
 * GBP_EINVAL beyond it, before reading any array. Indices are 32-bit; at
 * about 375 B of device memory per factor (FP32 state), the factor limit
 * lies above what one 288 GB GPU holds. */
#define GBP_MAX_BATCH_ITEMS 1073741824
gbp_status gbp_create_batch(int32_t n, const gbp_graph *graphs,
                            const gbp_camera *cameras,
                            const gbp_measurements *meas,
                            const gbp_options *opt, gbp_problem **out);

/* Relinearise (Section 5): beta < 0 selects every factor, otherwise the
 * factors whose stacked [mu_k; mu_m] lies farther than beta from their
 * linearisation point. The selected factors take the current means as their
 * linearisation point, with the Huber threshold last set on the problem;
 * the new linearisation is applied at the start of the next factor phase
 * (nothing in between depends on it). *n_relin (may be NULL) receives the
 * number selected; this call synchronises. GBP_EINVAL for a NaN beta. */
gbp_status gbp_relinearise(gbp_problem *p, double beta, int32_t *n_relin);

/* n synchronous iterations (Section 5): relinearisation check, factor
 * messages with damping `damping`, belief update. huber_k (px) is stored on
 * the problem and used by every relinearisation from now on. Asynchronous:
 * numerical failures are reported by the next synchronising call. */
gbp_status gbp_iterate(gbp_problem *p, int32_t n, double damping,
                       double huber_k);

/* Current beliefs in the caller's variable order (problem-major for
 * batches): means kf_mean [Nk][6], lm_mean [Nl][3]; information matrices
 * kf_info [Nk][6][6] and lm_info [Nl][3][3] when not NULL. Synchronises;
 * GBP_ENUMERIC if a belief failed to be positive definite since the last
 * check (that belief keeps its last good value). */
gbp_status gbp_beliefs(gbp_problem *p, double *kf_mean, double *lm_mean,
                       double *kf_info, double *lm_info);

/* Average reprojection error over all factors (every problem of a batch):
 * *are_all, *are_inlier_quadratic and *n_linear_regime may be NULL. */
gbp_status gbp_reproj_error(gbp_problem *p, double *are_all,
                            double *are_inlier_quadratic,
                            int32_t *n_linear_regime);

/* Full statistics of one problem of a batch (problem_index >= 0) or of the
 * whole graph (-1). Synchronises. */
gbp_status gbp_reproj_stats(gbp_problem *p, int32_t problem_index,
                            gbp_reproj *out);

/* Reference pixels (e.g. noise-free projections) and a mask selecting the
 * factors they apply to, in the caller's factor order; used for are_ref.
 * NULL clears the reference. */
gbp_status gbp_set_reference(gbp_problem *p, const double *z_ref,
                             const uint8_t *mask);

/* As gbp_iterate, and every log_every iterations records
 * {t, are_all, are_ref, n_linear, n_linear_ref} of every problem into a
 * device log; the log (n/log_every rows x n_problems x GBP_LOG_COLS doubles)
 * is copied to log_out at the end, with no host synchronisation in between. */
#define GBP_LOG_COLS 5
gbp_status gbp_iterate_logged(gbp_problem *p, int32_t n, double damping,
                              double huber_k, int32_t log_every,
                              double *log_out);

/* Heterogeneous factors (the outlook of Sections 9 and 10: factors from
 * further priors and sensors in the same graph). Appends n pairwise
 * difference factors between two keyframes (kind GBP_PAIR_KEYFRAMES, D = 6,
 * on the pose vector (omega, t)) or two landmarks (GBP_PAIR_LANDMARKS,
 * D = 3): x_b - x_a ~ N(z, diag(precision)^-1), e.g. a motion prior between
 * consecutive keyframes or a smoothness prior between neighbouring scene
 * points. a, b: [n] variable indices in the caller's order (problem-major
 * for batches; a != b); z, precision: [n][D] host arrays (precision > 0),
 * copied. The factors are linear and never relinearised; their messages
 * follow eqs. (messageeta), (messagelambda), are damped like the
 * measurement factors' (same d and damping mode, undamped for the first
 * `undamped_after_relin` updates after they were added; with a damping
 * model set they keep the constant damping) and start at zero;
 * they enter every later belief update. May be called at any clock and
 * repeatedly; synchronises. Their state lives in one extra device
 * allocation made here (outside a caller workspace). GBP_EINVAL for a bad
 * kind, index, a == b, non-finite z or non-positive precision, or more than
 * GBP_MAX_BATCH_ITEMS pairs between keyframes (odometry included) or between
 * landmarks in total (checked before the arrays are read); GBP_ESTATE on
 * a problem that has grown (gbp_add_keyframe), and afterwards
 * gbp_add_keyframe (and gbp_apply_depth_model, for landmark pairs) return
 * GBP_ESTATE. gbp_reset zeroes their messages and keeps them. */
#define GBP_PAIR_KEYFRAMES 0
#define GBP_PAIR_LANDMARKS 1
/* kind GBP_PAIR_ODOMETRY: an odometry factor between keyframes a and b
 * measuring the displacement of their camera centres in the world frame,
 * c_b - c_a ~ N(z, diag(precision)^-1) with c = -R(omega)^T t (z,
 * precision: [n][3]). Nonlinear: it is linearised at the current means at
 * every update and therefore, like any factor in the window that follows a
 * relinearisation, sends undamped messages. Same storage, rules and errors
 * as the keyframe difference factors. */
#define GBP_PAIR_ODOMETRY 2
gbp_status gbp_add_pair_factors(gbp_problem *p, int32_t kind, int32_t n,
                                const int32_t *a, const int32_t *b,
                                const double *z, const double *precision);

/* Incremental growth (Section 9.2) of a single (non-batched) problem:
 * append one keyframe with initial pose `pose` (NULL: no keyframe),
 * n_new_lm landmarks and n_new_f factors whose indices refer to the grown
 * variable sets (new keyframe = old count, new landmarks follow the old
 * ones). New factors are linearised at the current means; new variables get
 * automatic priors from the new factors and their own annealing clock.
 * A reference set with gbp_set_reference is dropped (set it again for the
 * grown factor set). GBP_ENOMEM when the capacity set at creation is
 * exceeded. */
gbp_status gbp_add_keyframe(gbp_problem *p, const double pose[6],
                            int32_t n_new_lm, const double *lm_init,
                            int32_t n_new_f, const int32_t *f_kf,
                            const int32_t *f_lm, const double *z);

/* ---- learned damping ------------------------------------------------------
 * The paper damps every message with one constant (Section 5, Section 8)
 * and names learned components as future work (Section 10). This library
 * replaces the constant by a per-factor value predicted by a small network
 * (16 features -> 64 -> 64 -> 2, ReLU) evaluated on the GPU every few
 * iterations; the network leaves the fixed points unchanged, since damping
 * does (Section 5). Parameter blob (GBP_MLP_PARAMS values): W1[64][16],
 * b1[64], W2[64][64], b2[64], W3[2][64], b3[2], row-major, output j of a
 * layer = b[j] + sum_i W[j][i] in[i]. Heads: damping d = 0.9 sigmoid(o0),
 * log-depth correction delta = 2.5 tanh(o1). Inference uses BF16 weights,
 * inputs and hidden activations (round to nearest even) with FP32 sums. */
#define GBP_MLP_PARAMS 5378
#define GBP_MLP_FEATURES 16

/* Per-factor damping model. `weights` (host, GBP_MLP_PARAMS BF16 bit
 * patterns, copied) switches it on; NULL restores the constant damping
 * passed to gbp_iterate. While on, every iteration whose clock t satisfies
 * t % every_k == 0 first evaluates the per-problem mean reprojection error,
 * the fallback monitor, the features (gbp_factor_features) and the network,
 * whose damping head replaces the constant damping of each factor outside
 * its undamped window. Fallback: a problem whose mean reprojection error
 * exceeds (1 + fallback_rise) x the best value seen since the model was set
 * (or since its last growth; with a plain-GBP judge, see
 * gbp_set_damping_judges, x the judge's error at the same iteration), or is
 * not finite, or one of whose beliefs failed, goes back to the constant
 * damping for good (fallback_rise <= -1: never; a
 * value in (-1, 0) switches every problem at the second evaluation). The
 * first call allocates about 116 bytes of device memory per factor of
 * capacity, owned by the problem. Errors: GBP_EINVAL for every_k outside
 * [1, 1000] or a NaN fallback_rise. Synchronises. */
gbp_status gbp_set_damping_model(gbp_problem *p, const uint16_t *weights,
                                 int32_t every_k, double fallback_rise);

/* Plain GBP as the judge of the learned damping (for batches). judge_of[i]
 * = j >= 0 names problem j of the batch as the judge of problem i: j must
 * hold the same problem (same graph, measurements and initial estimate) and
 * it runs the constant damping throughout; at every model evaluation problem
 * i goes back to the constant damping for good when its mean reprojection
 * error exceeds (1 + fallback_rise) x its judge's at the same iteration (in
 * place of the best-seen rule of gbp_set_damping_model). judge_of[i] = -1:
 * problem i keeps the best-seen rule; NULL: no judges. A judge cannot have a
 * judge. Kept across gbp_reset and gbp_set_damping_model. Errors:
 * GBP_ESTATE without a damping model, GBP_EINVAL for a judge index outside
 * the batch, equal to i, or itself judged. Synchronises. */
gbp_status gbp_set_damping_judges(gbp_problem *p, const int32_t *judge_of);

/* Restart: back to the state right after creation (every factor linearised
 * at the initial estimate, zero messages, beliefs = priors at clock 0, and
 * the damping model's history and fallback state cleared). Recorded
 * iteration graphs, the reference, the damping model and the tuning stay,
 * so a restarted run replays without re-recording. GBP_ESTATE after
 * gbp_add_keyframe. Synchronises. */
gbp_status gbp_reset(gbp_problem *p);

/* Learned initial depth (the second head of the damping model): for each
 * listed landmark (caller indices, host array; duplicates ignored) the
 * network is evaluated on every factor, and the landmark is moved along the
 * ray from the camera centre of its newest observing keyframe to
 * c + exp(mean log-depth head over its factors) (l - c); its prior mean moves
 * with it, and every one of its factors is relinearised at the new position
 * with zero messages (a fresh start for that landmark; GBP is insensitive to
 * the prior mean, Section 8). Meant for landmarks initialised at a guessed
 * depth a few iterations after they join (Section 9.2). Also advances the
 * feature history and rewrites the per-factor damping. GBP_ESTATE without a
 * model (gbp_set_damping_model), GBP_EINVAL for an index outside
 * [0, n_landmarks). Synchronises. */
gbp_status gbp_apply_depth_model(gbp_problem *p, const int32_t *landmarks,
                                 int32_t n);

/* Per-problem fallback state of the damping model (flags[n_problems]: 1 =
 * switched back to the constant damping; judges read 1). Synchronises. */
gbp_status gbp_fallback_flags(gbp_problem *p, int32_t *flags);

/* Features of the damping model, in the caller's factor order: computes the
 * 16 features of every factor from the current state, advances their
 * history (the message changes are taken since the previous evaluation)
 * and writes row i of out (device, [n][16] float) for factor idx[i]
 * (device int32). Rows of indices outside [0, n_factors) are NaN.
 * Features: 0 residual at the linearisation point / Huber threshold,
 * 1 Huber weight, 2 log(1 + residual / sigma), 3 updates since the last
 * linearisation / 10, 4 log(1 + distance from the linearisation point /
 * beta), 5-6 relative change of the keyframe- and landmark-side message
 * vectors, 7 relative change of the landmark-side message information,
 * 8 and 13 cosine of consecutive landmark- and keyframe-side message
 * changes, 9 log(depth / 5 m), 10-11 log degrees of landmark and keyframe,
 * 12 log trace of the landmark covariance / 10, 14 iteration / 300,
 * 15 log(1 + pixel shift of the landmark since its linearisation).
 * Synchronises. */
gbp_status gbp_factor_features(gbp_problem *p, const int32_t *idx, int32_t n,
                               float *out);

/* Messages of factors idx[i] (device int32, caller order) into out (device,
 * [n][16] float): S and g of the message to the keyframe (S = [[a b][b c]]
 * as a, b, c; g in the factor's 2-D measurement space), the same for the
 * landmark, the updates since the last linearisation, the factor's flags,
 * then J_k a_k and J_m a_m (2 each). The message to variable v in variable
 * space is information J_v^T S J_v and information vector
 * J_v^T (g + S J_v a_v), with J_v the factor's Jacobian block and a_v the
 * variable's initial estimate. Rows of indices outside [0, n_factors) are
 * NaN. Synchronises. */
gbp_status gbp_factor_messages(gbp_problem *p, const int32_t *idx, int32_t n,
                               float *out);

/* Network inference on caller buffers (all device pointers): x [n][16]
 * float, 16-byte aligned (each row is read as 16-byte vectors; a misaligned
 * x is GBP_EINVAL), weights GBP_MLP_PARAMS BF16, d_out [n] damping head,
 * delta_out [n] log-depth head (may be NULL). Asynchronous on `stream`
 * (hipStream_t, NULL = default stream). Errors (GBP_EINVAL, GBP_EDEVICE)
 * leave their text in gbp_last_error(NULL). */
gbp_status gbp_mlp_infer(const uint16_t *weights, const float *x, int32_t n,
                         float *d_out, float *delta_out, void *stream);

/* The same with the features already stored as BF16 bit patterns, x_bf16
 * [n][16] (device, 16-byte aligned): half the bytes per row; the network
 * rounds its FP32 inputs to BF16 (nearest even) anyway, so features rounded
 * that way give bit for bit the outputs of gbp_mlp_infer. Errors as
 * gbp_mlp_infer. */
gbp_status gbp_mlp_infer_bf16(const uint16_t *weights, const uint16_t *x_bf16,
                              int32_t n, float *d_out, float *delta_out,
                              void *stream);

/* Device workspace bytes of gbp_mlp_train_step for batches up to max_batch. */
gbp_status gbp_mlp_train_workspace_bytes(int32_t max_batch, size_t *bytes);

/* One training step of the network on caller buffers (all device pointers).
 * Data: x [n_rows][16], targets y [n_rows][2] (damping, log-depth), sample
 * weights mask [n_rows][2]; the batch is rows batch_idx[0..n_batch) (an
 * index outside [0, n_rows) counts as a zero-weight sample). Loss
 * (written to loss_out[0]): (1/n_batch) sum over the batch of
 * mask0 (d - y0)^2 + mask1 (delta - y1)^2, with the forward pass of
 * gbp_mlp_infer evaluated at the BF16 rounding of theta (FP32 master
 * weights, GBP_MLP_PARAMS) and back-propagated in FP32; its gradient goes to
 * grad_out [GBP_MLP_PARAMS]. step >= 1: then one Adam step (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias correction for step `step`, learning rate lr)
 * updates theta, adam_m, adam_v and writes the BF16 copy weights_bf16.
 * step == 0: gradient and loss only (adam_m, adam_v, weights_bf16 may be
 * NULL). Sums are in a fixed order: the result is deterministic.
 * Asynchronous on `stream`. */
gbp_status gbp_mlp_train_step(const float *x, const float *y, const float *mask,
                              int32_t n_rows, const int32_t *batch_idx,
                              int32_t n_batch, float *theta, float *adam_m,
                              float *adam_v, uint16_t *weights_bf16, float lr,
                              int32_t step, float *grad_out, float *loss_out,
                              void *workspace, size_t workspace_bytes,
                              void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc): gbp_mlp_train_step without a workspace. Same arguments,
 * results and errors as gbp_mlp_train_step (bitwise the same results); the
 * partial gradients live in a fixed device array inside the library of
 * GBP_MLP_STATIC_MAX_BATCH samples' worth (about 5.5 MB, held on each GPU
 * the library runs on until the process ends). n_batch above
 * GBP_MLP_STATIC_MAX_BATCH: GBP_EINVAL. `stream` (NULL = default stream)
 * must belong to the current device. Allocates nothing; the first call on a
 * device looks up the array's address there. Every call on one GPU shares
 * that array: calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller. */
#define GBP_MLP_STATIC_MAX_BATCH 8192
gbp_status gbp_mlp_train_step_static(const float *x, const float *y,
                                     const float *mask, int32_t n_rows,
                                     const int32_t *batch_idx, int32_t n_batch,
                                     float *theta, float *adam_m, float *adam_v,
                                     uint16_t *weights_bf16, float lr,
                                     int32_t step, float *grad_out,
                                     float *loss_out, void *stream);

/* Per-phase timing (the compute phases of one iteration, Section 7 and
 * Fig. 3): runs n iterations with each phase launched separately and
 * bracketed by HIP events on the problem's stream, then writes the average
 * milliseconds per launch of {relinearisation check, relinearisation of the
 * due factors, factor messages + keyframe beliefs, landmark beliefs,
 * reprojection statistics} to ms_out[0..4], and to ms_out[5] the average
 * duration of the keyframe factor kernel alone (events recorded by the
 * driver at the kernel's start and end). The iterations are real: the
 * state advances by n. Synchronises. */
gbp_status gbp_phase_times(gbp_problem *p, int32_t n, double damping,
                           double huber_k, double *ms_out);

/* Number of factors relinearised in the most recent iteration (the subset
 * of factors that relinearise each iteration, Section 7, Fig. 3).
 * Synchronises. */
gbp_status gbp_counters(gbp_problem *p, int64_t *relinearisations);

/* Autotuner: picks the workgroup sizes of the keyframe factor kernel and of
 * the landmark belief kernel (64/128/256 each, with 4 lanes per landmark),
 * then the lanes per landmark (2/4/8), then whether the keyframe solves run
 * in the first workgroups of the landmark-belief launch or in a launch of
 * their own (same arithmetic, bit for bit), by timing n_iters iterations of
 * every candidate with HIP events on this problem, then the relinearisation
 * queue segments per workgroup (1/2/4) by timing n_iters relinearisation
 * launches on a synthetic queue holding every 11th factor (about the share
 * due per iteration at steady state); the device state is restored after
 * each candidate (the problem's results are unchanged). The choice is
 * cached in the text file cache_path (may be NULL: no cache), keyed by GPU
 * architecture, precision and size bucket; a cached entry is used without
 * timing (entries of an older format are ignored). chosen[5] (may be NULL)
 * receives the two sizes, the lane count, the segment count and the
 * keyframe-solve placement (1: inside the landmark-belief launch). Allocates
 * a temporary copy of the workspace. Synchronises. */
gbp_status gbp_autotune(gbp_problem *p, int32_t n_iters, const char *cache_path,
                        int32_t *chosen);

/* Sizes: keyframes, landmarks, factors, problems, completed iterations. */
gbp_status gbp_sizes(const gbp_problem *p, int32_t *n_keyframes,
                     int32_t *n_landmarks, int32_t *n_factors,
                     int32_t *n_problems, int32_t *t);

/* Message describing the last error on this problem (never NULL). */
const char *gbp_last_error(const gbp_problem *p);

void gbp_destroy(gbp_problem *p);

#ifdef __cplusplus
}
#endif
#endif /* GBP_H */
