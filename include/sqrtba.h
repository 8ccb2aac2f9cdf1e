/*
 * sqrtba.h -- C ABI of libsqrtba.so: square-root bundle adjustment on one
 * AMD Instinct MI355X (gfx950), FP32, after Demmel, Sommer, Cremers, Usenko,
 * "Square Root Bundle Adjustment for Large-Scale Reconstruction" (CVPR 2021).
 * The same calls in double precision (the method's FP64 variant) are declared
 * in sqrtba64.h and exported by libsqrtba64.so.
 *
 * The calls follow the problem statement of the paper (Sec. 4): cameras,
 * landmarks and observations define the energy E = sum |r_ij|^2
 * (eq. ba_energy); one Levenberg-Marquardt step is linearize (Sec. 4.1,
 * eq. linearized_residual), marginalize landmarks by QR (Sec. 4.3 and 5.2),
 * damp (Sec. 5.3), solve the reduced camera system with PCG (Sec. 5.4,
 * eq. cg_mult), back-substitute (eq. backsub_nm), and update (Sec. 6.1).
 *
 * Conventions shared by every call
 *  - Every function returns a sqrtba_status; no C++ exception crosses the ABI.
 *    On error the context state is unchanged and sqrtba_last_error() explains.
 *  - Array arguments are HOST pointers unless stated otherwise (the *_device
 *    calls take DEVICE pointers for the problem's inputs and state); the
 *    library copies inputs during the call and writes outputs before
 *    returning, so the caller keeps ownership of all its buffers.  Device memory is owned by the
 *    context (allocated by the library, or a caller-provided workspace bound
 *    with sqrtba_bind_workspace) and released by sqrtba_destroy.
 *  - All kernels run on the HIP stream given at creation (NULL = default).
 *    Calls that return values synchronize that stream.
 *  - A context may hold several independent problems (a batch, see
 *    sqrtba_set_problems).  "[P]" marks an array with one entry per problem;
 *    a single problem is the batch with P = 1, so a pointer to one scalar is a
 *    valid [P] array.
 *  - Cameras are the 9-vector (w, t, f, k1, k2) of the BAL "Snavely" model
 *    (Sec. 6.2): P = R(w) X + t, p = -P_xy / P_z,
 *    pixel = f (1 + k1 |p|^2 + k2 |p|^4) p, relative to the image centre.
 *    Internally R is a matrix updated on the left, R <- Exp(dw) R.
 *  - A landmark with fewer than two observations and a camera with no
 *    observation are not errors: they are inactive and held fixed (Sec. 6.2
 *    removes such landmarks in preprocessing).
 *  - Not thread-safe: one context must not be used from two threads at once.
 */
#ifndef SQRTBA_H
#define SQRTBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sqrtba_ctx sqrtba_ctx;

typedef enum {
  SQRTBA_OK = 0,
  SQRTBA_E_INVALID = -1,       /* bad argument or invalid input data */
  SQRTBA_E_OOM = -2,           /* device or host allocation failed, or workspace too small */
  SQRTBA_E_HIP = -3,           /* a HIP runtime call failed */
  SQRTBA_E_STATE = -4,         /* call out of order (e.g. solve before marginalize) */
  SQRTBA_E_NONFINITE = -5,     /* non-finite input value */
  SQRTBA_E_UNSUPPORTED = -6    /* e.g. a landmark with more observations than SQRTBA_MAX_OBS_PER_LANDMARK */
} sqrtba_status;

/* Largest number of observations of one landmark the stored-block kernels accept. */
#define SQRTBA_MAX_OBS_PER_LANDMARK 512

/* Per-problem outcome of a PCG solve and of the LM loop. */
enum {
  SQRTBA_PCG_CONVERGED = 0,    /* |r_k| <= tol |r_0| (unpreconditioned) */
  SQRTBA_PCG_MAX_ITERS = 1,
  SQRTBA_PCG_BREAKDOWN = 2,    /* p^T A p <= 0 or a non-finite value; last x kept */
  SQRTBA_PCG_ZERO_RHS = 3,
  SQRTBA_PCG_INACTIVE = 4
};
enum {
  SQRTBA_LM_MAX_ITERS = 0,
  SQRTBA_LM_FUNC_TOL = 1,      /* accepted step with (E_old - E_new) / E_old < func_tol */
  SQRTBA_LM_LAMBDA_MAX = 2,    /* damping reached lambda_max */
  SQRTBA_LM_NONFINITE = 3
};

typedef struct {
  double lambda0;        /* initial LM damping, 1e-4 (Sec. 6.1) */
  double lambda_min;     /* 1e-16 */
  double lambda_max;     /* 1e32; reaching it ends the solve */
  double accept_ratio;   /* accept a step iff rho > accept_ratio, 1e-3 */
  int32_t max_lm_iters;  /* every attempt counts, 50 (Sec. 6.1) */
  double func_tol;       /* relative function tolerance, 1e-6 (Sec. 6.1) */
  int32_t pcg_max_iters; /* 500, no minimum (Sec. 6.1) */
  double pcg_rel_tol;    /* stop when |r_k| / |r_0| <= tol, 1e-6 */
  int32_t pcg_check_every; /* host checks convergence every n iterations (device flags stop work in between), 8 */
  int32_t use_graph;     /* capture chunks of PCG iterations in a HIP graph, 1 */
  double pcg_forcing_eta; /* 0 (default): PCG stops on pcg_rel_tol or pcg_max_iters only.  > 0:
                             it also stops at the first iteration i >= 1 with
                             i (Q_i - Q_{i-1}) / Q_i < eta, Q the quadratic model of the
                             reduced system at the iterates (tracked as Q_{i+1} = Q_i -
                             alpha_i r_i.z_i / 2): the truncated-Newton test of Nash and Sofer
                             (1990), read as the "same forcing sequence as Ceres" of Sec. 6.1,
                             where eta = 0.1 */
  int32_t landmark_blocks; /* 0 (default): explicit landmark blocks, the 2k x 9k rows
                              [Q2^T J_p; damping rows] stored per landmark (Sec. 5.1).
                              1: implicit blocks: only the pose Jacobian rows and the thin
                              factor Q1 (24 floats per observation) are stored; the product
                              and everything else use B^T B = J_p^T (I - Q1 P Q1^T) J_p with
                              P = R1 (R1^T R1 + lambda I)^-1 R1^T, the same reduced system
                              (eq. red_H) at O(k) memory and traffic per landmark.
                              2: the explicit Schur complement in FP32, the comparator of the
                              paper's explicit solver (Sec. 4.2, eq. red_normal_eq): per
                              landmark H_ll, b_l and G = J_p^T J_l from the normal equations,
                              and H_pp - sum G (H_ll + lambda I)^-1 G^T assembled as 9 x 9
                              blocks per camera pair at every damp (O(sum k^2) host
                              bookkeeping, SQRTBA_E_UNSUPPORTED beyond 2^30 pair
                              contributions); the same PCG, preconditioner and LM loop.
                              Chosen before the workspace is sized; sqrtba_set_options
                              refuses to change it after upload (SQRTBA_E_STATE). */
  double huber_delta;    /* 0 (default): squared loss, E = sum |r_o|^2.  > 0: the Huber loss of
                            Sec. 6.2 with this parameter in pixels, applied by IRLS: per
                            observation s = |r_o|^2, E = sum rho(s) with rho(s) = s for
                            s <= delta^2 and 2 delta sqrt(s) - delta^2 beyond, and at every
                            linearization the observation's residual and Jacobian rows are
                            scaled by sqrt(rho'(s)) = sqrt(min(1, delta / |r_o|)).  Costs,
                            reports and histories are then robust costs; the model decrease is
                            the reweighted linear model's. */
  int32_t pcg_test_kernel; /* where the PCG convergence test runs (the result is the same bit for
                              bit): 0 in the per-camera kernel after the next product, which is
                              wasted once the test succeeds (one product per solve); 1 in a
                              kernel of its own after each update, which skips that product at
                              the cost of one small launch per iteration; -1 (default): 1 when
                              the product's algorithmic bytes over the problems of the solve
                              are at least 1 GiB, else 0 */
} sqrtba_options;

typedef struct {
  double initial_cost;
  double final_cost;
  int32_t iterations;    /* LM attempts, accepted or not */
  int32_t accepted;
  int32_t total_pcg_iters;
  int32_t status;        /* SQRTBA_LM_* */
  double solve_seconds;  /* wall time from loop start until this problem finished */
  double time_to_tol;    /* seconds until cost <= tol_cost, or -1 (set by sqrtba_lm_solve_tracked) */
} sqrtba_lm_report;

typedef struct {
  int32_t iter;
  int32_t accepted;
  int32_t pcg_iters;
  int32_t pcg_status;
  double lambda;
  double cost;           /* cost before the attempt */
  double new_cost;       /* cost at the tentative state */
  double model_decrease;
  double rel_res;
  double t_seconds;      /* wall time since the start of the LM loop, at the end of the attempt */
} sqrtba_lm_record;

/* Library version, for ABI checks. */
int32_t sqrtba_version(void);

/* Fill *opt with the defaults listed above. */
void sqrtba_default_options(sqrtba_options* opt);

/* Create a context on the current HIP device.  hip_stream is a hipStream_t
 * (NULL: the default stream).  opt may be NULL for defaults. */
int32_t sqrtba_create(sqrtba_ctx** out, const sqrtba_options* opt, void* hip_stream);

/* Replace the options of an existing context (same validation as create:
 * SQRTBA_E_INVALID on negative limits, lambda0 <= 0, pcg_check_every < 1, a
 * negative or non-finite pcg_forcing_eta or huber_delta; the context is then
 * unchanged).
 * Takes effect from the next call. */
int32_t sqrtba_set_options(sqrtba_ctx* ctx, const sqrtba_options* opt);

/* Free every resource of ctx (NULL is allowed). */
void sqrtba_destroy(sqrtba_ctx* ctx);

/* Text of the last error of ctx; valid until the next call on ctx. */
const char* sqrtba_last_error(const sqrtba_ctx* ctx);

/* Optional, before sqrtba_set_cameras: split the context into n_problems
 * independent problems.  cam_off and pt_off are CSR offsets of length
 * n_problems + 1 (starting at 0) over the camera and landmark arrays;
 * every observation must link a camera and a landmark of the same problem. */
int32_t sqrtba_set_problems(sqrtba_ctx* ctx, int32_t n_problems, const int64_t* cam_off, const int64_t* pt_off);

/* Cameras: n_cams x 9 floats, row-major, BAL order (w0 w1 w2 t0 t1 t2 f k1 k2). */
int32_t sqrtba_set_cameras(sqrtba_ctx* ctx, int64_t n_cams, const float* params);

/* Landmarks: n_points x 3 floats, row-major. */
int32_t sqrtba_set_landmarks(sqrtba_ctx* ctx, int64_t n_points, const float* xyz);

/* Observations: camera index, landmark index and pixel (u, v) each.  Sorts
 * them by (landmark, camera) (the landmark blocks of Sec. 5.1), builds the
 * CSR bookkeeping and checks them.  Errors: an index out of range, a
 * duplicate (camera, landmark) pair, an observation linking two problems
 * (SQRTBA_E_INVALID); a non-finite pixel (SQRTBA_E_NONFINITE); a landmark with
 * more than SQRTBA_MAX_OBS_PER_LANDMARK observations (SQRTBA_E_UNSUPPORTED). */
int32_t sqrtba_set_observations(sqrtba_ctx* ctx, int64_t n_obs, const int32_t* cam, const int32_t* pt,
                                const float* uv);

/* The three calls above with DEVICE pointers (e.g. torch.Tensor.data_ptr() of
 * contiguous CUDA tensors, same layouts and element types).  The library
 * copies the arrays to the host on the context's stream (the bookkeeping of
 * set_observations and the rotation conversion of set_cameras run there) and
 * then behaves exactly like the host-pointer call, errors included; the
 * caller keeps ownership.  A pointer that HIP does not report as device (or
 * managed) memory is SQRTBA_E_INVALID. */
int32_t sqrtba_set_cameras_device(sqrtba_ctx* ctx, int64_t n_cams, const float* params);
int32_t sqrtba_set_landmarks_device(sqrtba_ctx* ctx, int64_t n_points, const float* xyz);
int32_t sqrtba_set_observations_device(sqrtba_ctx* ctx, int64_t n_obs, const int32_t* cam, const int32_t* pt,
                                       const float* uv);

/* Device bytes the context needs once cameras, landmarks and observations are set. */
int32_t sqrtba_workspace_bytes(const sqrtba_ctx* ctx, uint64_t* bytes);

/* Use caller-owned DEVICE memory (at least sqrtba_workspace_bytes, 256-byte
 * aligned) instead of allocating; it must outlive the context.  Uploads the
 * problem.  Without this call the first compute call allocates and uploads. */
int32_t sqrtba_bind_workspace(sqrtba_ctx* ctx, void* device_ptr, uint64_t bytes);

/* Problems taking part in the following calls (mask[P], 1 = active).
 * All problems are active after upload. */
int32_t sqrtba_set_active(sqrtba_ctx* ctx, const uint8_t* mask);

/* Kernel (a): residuals at the current state, cost[P] (may be NULL), and the
 * unit-norm column scaling of the camera columns (Sec. 5.4). */
int32_t sqrtba_linearize(sqrtba_ctx* ctx, double* cost);

/* Kernel (b): for each landmark, linearize its observations, scale its
 * Jacobian columns to unit norm, QR-factor J_l with three Householder
 * reflections (Sec. 5.2) and store Q^T [J_p | r] as its landmark block
 * (Sec. 5.1): the top three rows for back-substitution and the 2k-3
 * nullspace rows of the reduced camera system (eq. reduced). */
int32_t sqrtba_marginalize(sqrtba_ctx* ctx);

/* Landmark damping (Sec. 5.3): fold sqrt(lambda) I into each landmark block
 * with six Givens rotations, starting from the stored undamped rows each time,
 * so a new lambda after a rejected step needs no new QR.  lambda[P] > 0. */
int32_t sqrtba_damp(sqrtba_ctx* ctx, const double* lambda);

/* Block-Jacobi preconditioner and right-hand side from the damped blocks,
 * then PCG on the reduced camera system with the matrix-free product
 * (B^T B + lambda I) v (Sec. 5.4, eq. cg_mult), from x0 = 0.  iters[P],
 * rel_res[P] and pcg_status[P] (SQRTBA_PCG_*) may be NULL. */
int32_t sqrtba_solve(sqrtba_ctx* ctx, int32_t* iters, double* rel_res, int32_t* pcg_status);

/* Back-substitution of every landmark (eq. backsub_nm with the damped
 * factors) and the decrease predicted by the undamped linear model,
 * model_decrease[P] (may be NULL). */
int32_t sqrtba_back_substitute(sqrtba_ctx* ctx, double* model_decrease);

/* Tentative state x (+) dx and its cost new_cost[P] (may be NULL). */
int32_t sqrtba_update(sqrtba_ctx* ctx, double* new_cost);

/* Keep (accept[P] = 1) or drop the tentative state of each active problem. */
int32_t sqrtba_commit(sqrtba_ctx* ctx, const uint8_t* accept);

/* The whole Levenberg-Marquardt loop (Sec. 6.1) for every problem at once,
 * report[P] may be NULL.  With tol_cost[P] (may be NULL) the report's
 * time_to_tol records when each problem's cost first fell to tol_cost. */
int32_t sqrtba_lm_solve(sqrtba_ctx* ctx, sqrtba_lm_report* report);
int32_t sqrtba_lm_solve_tracked(sqrtba_ctx* ctx, const double* tol_cost, sqrtba_lm_report* report);

/* Per-attempt history of problem `problem` from the last LM solve. */
int32_t sqrtba_get_lm_history(const sqrtba_ctx* ctx, int32_t problem, sqrtba_lm_record* out, int32_t capacity,
                              int32_t* n_records);

/* Current state: n_cams x 9 (BAL order; w from the rotation matrix, host FP64) and n_points x 3. */
int32_t sqrtba_get_cameras(sqrtba_ctx* ctx, float* params);
int32_t sqrtba_get_landmarks(sqrtba_ctx* ctx, float* xyz);
/* The same into caller-owned DEVICE arrays (n_cams x 9, n_points x 3), written on
 * the context's stream, which is synchronized before returning. */
int32_t sqrtba_get_cameras_device(sqrtba_ctx* ctx, float* params);
int32_t sqrtba_get_landmarks_device(sqrtba_ctx* ctx, float* xyz);

/* ---- inspection exports for tests (small problems) ---- */

/* Canonical bookkeeping: obs_perm[n_active] (input index of each active
 * observation sorted by (landmark, camera)), lm_off[n_points + 1],
 * lm_active[n_points], cam_active[n_cams]; *n_active receives the count
 * (call with NULL arrays first to size them). */
int32_t sqrtba_debug_bookkeeping(const sqrtba_ctx* ctx, int64_t* n_active, int64_t* obs_perm, int64_t* lm_off,
                                 uint8_t* lm_active, uint8_t* cam_active);

/* Kernel (a)'s per-observation values at the current state, in obs_perm
 * order: r[n_active x 2], Jp[n_active x 2 x 9], Jl[n_active x 2 x 3]
 * (unscaled; any may be NULL). */
int32_t sqrtba_debug_linearization(sqrtba_ctx* ctx, float* r, float* Jp, float* Jl);

/* Column scales of the last linearize/marginalize: s_cam[n_cams x 9], s_pt[n_points x 3]. */
int32_t sqrtba_debug_scales(sqrtba_ctx* ctx, float* s_cam, float* s_pt);

/* Damped reduced-camera-system products (B^T B + lambda I) v in scaled
 * coordinates for m vectors v[m x 9 n_cams] -> out[m x 9 n_cams]; and the
 * right-hand side b~ = sum B^T (Q2^T r), rhs[9 n_cams].  Needs damp. */
int32_t sqrtba_debug_rcs_matvec(sqrtba_ctx* ctx, int32_t m, const float* v, float* out);
int32_t sqrtba_debug_rhs(sqrtba_ctx* ctx, float* rhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the product of
 * sqrtba_debug_rcs_matvec for ONE vector, with DEVICE pointers v[9 n_cams] and
 * out[9 n_cams] (scaled coordinates, out = (B^T B + lambda I) v), enqueued on the
 * context's stream without synchronizing.  It allocates nothing: the product's
 * scaled input (12 elements per camera), per-observation outputs and row-block
 * partials go to a static device array
 * of SQRTBA_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends (looked up at sqrtba_create).  Every call on a GPU shares
 * that array: calls that overlap on one GPU (two streams, two contexts, two
 * threads) race.  Explicit landmark blocks only (SQRTBA_E_UNSUPPORTED for the
 * other forms); a problem whose scratch exceeds the array is
 * SQRTBA_E_UNSUPPORTED.  Needs damp. */
#define SQRTBA_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t sqrtba_rcs_matvec_noalloc(sqrtba_ctx* ctx, const float* v, float* out);

/* Inverse block-Jacobi blocks [n_cams x 81] of the last solve. */
int32_t sqrtba_debug_precond(sqrtba_ctx* ctx, float* minv);

/* Landmark block of landmark `pt` after marginalize (and damp): *k receives
 * its observation count (0: inactive).  If out != NULL it receives
 * (2k+3) x (9k+4) floats: rows 0..2 the undamped top rows
 * [Q1^T J_p | R1 | Q1^T r], rows 3..2k+2 the B rows [B | 0 | rho] (the 2k-3
 * nullspace rows, then the 3 damping rows written by damp); pose columns are
 * unscaled, landmark columns are scaled.  If factors != NULL it receives 24
 * floats: R1 upper (6, row-major), Q1^T r (3), damped R upper (6), damped
 * Q1^T r (3), landmark column scales (3), lambda of the last damp (1), 0, 0.
 * With implicit landmark blocks there are no block rows: out must be NULL
 * (else SQRTBA_E_UNSUPPORTED); factors as above.  With the explicit Schur
 * complement (landmark_blocks = 2) out must be NULL too, and factors holds the
 * scaled H_ll upper (6), the scaled b_l (3), unused (9), the landmark column
 * scales (3), lambda (1), 0, 0. */
int32_t sqrtba_debug_block(sqrtba_ctx* ctx, int64_t pt, int32_t* k, float* out, float* factors);

/* Solution of the last solve/back-substitution: scaled pose increment
 * dxp[9 n_cams] and unscaled landmark increment dxl[n_points x 3]. */
int32_t sqrtba_debug_solution(sqrtba_ctx* ctx, float* dxp_scaled, float* dxl);

/* Replace the scaled pose increment (for testing back-substitution). */
int32_t sqrtba_debug_set_pose_increment(sqrtba_ctx* ctx, const float* dxp_scaled);

/* ---- learned block preconditioner (the project's extension; not in the paper) ----
 *
 * Per camera, an MLP 64 -> 128 -> 128 -> 81 (tanh; bfloat16 weights, FP32
 * accumulation) maps 64 features of the damped 9x9 block-Jacobi block
 * P = L L^T (log diagonal, correlations, log(lambda / P_aa), log lambda, the
 * camera's observation and covisibility counts, mean and max log k, log of the
 * mean diagonal) to E; the inverse block used by PCG is M^-1 = C C^T with
 * C = L^-T (I + 0.1 tanh(tril E)), symmetric positive definite by
 * construction, and exactly P^-1 when E = 0.  Parameters are one FP32 array
 * [W1 (64x128), b1, W2 (128x128), b2, W3 (128x81), b3], row-major [in][out].
 * Training minimizes the mean over traced PCG pairs (p, q = A p) and cameras i
 * of |M_i^-1 q_i - p_i|^2 / |p_i|^2 with Adam, on the GPU. */

/* Number of network parameters (35281). */
int32_t sqrtba_mlp_num_params(void);

/* Initialize the network (Xavier-uniform hidden layers, zero output layer:
 * block-Jacobi behaviour) from a seed; resets the optimizer. */
int32_t sqrtba_mlp_init(sqrtba_ctx* ctx, uint64_t seed);

/* Set / get the FP32 parameters (host arrays of sqrtba_mlp_num_params()). */
int32_t sqrtba_mlp_set_params(sqrtba_ctx* ctx, const float* params);
int32_t sqrtba_mlp_get_params(sqrtba_ctx* ctx, float* params);

/* Preconditioner of subsequent solves: 0 = block-Jacobi (default), 1 = learned.
 * In learned mode a problem whose PCG does not reach the tolerance within 1.5x
 * the iterations of its last block-Jacobi solve (or breaks down) is solved again
 * from scratch with block-Jacobi, so the tolerance and the result of the solve
 * are those of the plain method.  The one exception: when the last block-Jacobi
 * solve of that problem also ended at pcg_max_iters, a learned run that ends
 * there too is kept (status MAX_ITERS), since a restart could not reach the
 * tolerance either. */
int32_t sqrtba_set_preconditioner(sqrtba_ctx* ctx, int32_t mode);

/* Record PCG traces for training: features and factors of up to max_solves
 * solves and (p, A p) of their first iters_per_solve iterations (device
 * memory; (0, 0) frees it).  Tracing runs PCG without graph capture. */
int32_t sqrtba_pcg_trace(sqrtba_ctx* ctx, int32_t max_solves, int32_t iters_per_solve);
int32_t sqrtba_trace_size(const sqrtba_ctx* ctx, int32_t* n_solves, int32_t* n_records);

/* steps Adam steps (learning rate lr) on minibatches of `batch` (record, camera)
 * samples drawn uniformly from the traces with a seeded generator; losses[steps]
 * (may be NULL) receives each minibatch's mean loss before its step.  lr = 0
 * only evaluates the loss on the same seeded minibatches (no update); lr < 0
 * or NaN is SQRTBA_E_INVALID. */
int32_t sqrtba_mlp_train(sqrtba_ctx* ctx, int32_t steps, int32_t batch, double lr, uint64_t seed, double* losses);

/* Loss and gradient at the current parameters for n explicit samples:
 * feats[n x 64], lfac[n x 45] (lower Cholesky factors, packed rows), p[n x 9],
 * q[n x 9]; *loss is the mean loss, grad[num_params] its gradient (may be NULL). */
int32_t sqrtba_mlp_eval(sqrtba_ctx* ctx, int32_t n, const float* feats, const float* lfac, const float* p,
                        const float* q, double* loss, float* grad);

/* Counters of learned-mode solves, fallbacks to block-Jacobi and the PCG
 * iterations those fallbacks discarded. */
int32_t sqrtba_learned_stats(const sqrtba_ctx* ctx, int64_t* learned_solves, int64_t* fallbacks,
                             int64_t* wasted_iters);

/* Inspection: per-camera features [n_cams x 64] and factors [n_cams x 45] of the
 * damped blocks, and the learned inverse blocks [n_cams x 81].  Need damp. */
int32_t sqrtba_debug_features(sqrtba_ctx* ctx, float* feats, float* lfac);
int32_t sqrtba_debug_learned_precond(sqrtba_ctx* ctx, float* minv);

/* ---- measurement and state snapshots ---- */

/* Stages timed by the profiler (HIP events on the context stream). */
enum {
  SQRTBA_STAGE_LINEARIZE = 0,   /* kernel (a): cost and column scales */
  SQRTBA_STAGE_MARGINALIZE = 1, /* kernel (b): per-landmark QR into landmark blocks */
  SQRTBA_STAGE_DAMP = 2,        /* Givens landmark damping */
  SQRTBA_STAGE_PRECOND = 3,     /* block-Jacobi blocks, right-hand side, PCG start */
  SQRTBA_STAGE_MATVEC = 4,      /* kernel (c): one PCG product over all landmark blocks */
  SQRTBA_STAGE_PCG_VECTOR = 5,  /* unused (vector work is inside the PCG loop) */
  SQRTBA_STAGE_BACKSUB = 6,     /* back-substitution and model decrease */
  SQRTBA_STAGE_UPDATE = 7,      /* tentative update and its cost */
  SQRTBA_NUM_STAGES = 8
};

/* Accumulated per-stage figures since profiling was enabled: total
 * milliseconds, number of timed executions, algorithmic bytes (the method's
 * own traffic: for MATVEC 4 (18k^2 + 9k) per landmark and product, for
 * MARGINALIZE 4 (2k (9k+1) + 12) + 12k + 16 per landmark) and units
 * (landmark blocks processed). */
typedef struct {
  double ms[SQRTBA_NUM_STAGES];
  int64_t launches[SQRTBA_NUM_STAGES];
  double bytes[SQRTBA_NUM_STAGES];
  int64_t units[SQRTBA_NUM_STAGES];
} sqrtba_profile;

/* Enable (on != 0) or disable the profiler; either way the counters restart. */
int32_t sqrtba_profile_enable(sqrtba_ctx* ctx, int32_t on);
int32_t sqrtba_profile_get(const sqrtba_ctx* ctx, sqrtba_profile* out);

/* Save the current camera and landmark state on the device, and restore it
 * (restoring invalidates the linearization).  For repeated solves from one
 * start and for checkpoint/resume of the LM state. */
int32_t sqrtba_save_state(sqrtba_ctx* ctx);
int32_t sqrtba_restore_state(sqrtba_ctx* ctx);

/* ---- launch shapes of the PCG product and their autotuner ---- */

/* The product runs size-bucketed kernels (landmarks by observation count k).
 * These are its tunable bucket edge, launch shapes and load policy.  None of them changes
 * the arithmetic except rows_min_k and huge_rows, which decide how the rows
 * of the largest blocks are grouped before their partial products are added. */
typedef struct {
  int32_t rows_min_k;     /* bucket edge: landmarks with k >= rows_min_k (114, 61 or 29)
                             take the row-block kernel, the others with k >= 29 the
                             four-wavefront landmark kernel */
  int32_t huge_rows;      /* rows per workgroup of the row-block kernel: 64, 128, 256,
                             512 or 1024 (1024: one workgroup per landmark, no partials) */
  int32_t huge_side;      /* 1: the row-block kernel runs on a second stream,
                             concurrently with the rest of the product */
  int32_t large_separate; /* 1: the four-wavefront landmarks get a launch of their own
                             (the small-class kernel then needs fewer registers) */
  int32_t small_rows;     /* rows per batch for k <= 28: 4 or 8 */
  int32_t persist_wgs;    /* 0: one workgroup per block of small landmarks; 1024, 2048
                             or 4096: a persistent launch of that many workgroups */
  int32_t stream_loads;   /* 0..3, two bits; bit 0 (1): the row-block and four-wavefront
                             landmark kernels read the blocks with non-temporal loads (no
                             cache allocation); bit 1 (2): so does the kernel of the
                             landmarks with k <= 28.  They help when the blocks are much
                             larger than the last-level cache and hurt when they fit in
                             it; 0: ordinary loads everywhere */
} sqrtba_tuning;

typedef struct {
  sqrtba_tuning shape;
  double ms;              /* mean milliseconds per product */
} sqrtba_tuning_trial;

/* Current shapes; set_tuning rejects values outside the lists above with
 * SQRTBA_E_INVALID.  Both need the problem uploaded (any solver call uploads
 * it; sqrtba_workspace_bytes/bind_workspace must have been satisfied). */
int32_t sqrtba_get_tuning(sqrtba_ctx* ctx, sqrtba_tuning* out);
int32_t sqrtba_set_tuning(sqrtba_ctx* ctx, const sqrtba_tuning* shape);

/* Time the product on the uploaded problem under candidate shapes and keep the
 * fastest: a coordinate search over the fields in the order above, each
 * candidate timed over `reps` products (<= 0: 10) with HIP events on the
 * context stream.  The timing does not depend on the values in the landmark
 * blocks, so this may run right after upload; it overwrites only scratch
 * (the product outputs).  best (may be NULL) receives the chosen shapes,
 * trials (may be NULL) up to max_trials records and *n_trials (may be NULL)
 * the number of candidates timed.  The shapes belong to the explicit-block
 * product; with implicit landmark blocks only the current shape is timed (one
 * trial) and kept. */
int32_t sqrtba_autotune(sqrtba_ctx* ctx, int32_t reps, sqrtba_tuning* best, sqrtba_tuning_trial* trials,
                        int32_t max_trials, int32_t* n_trials);

/* Mean milliseconds of one PCG product (kernel (c), current shapes) over reps
 * back-to-back launches on the resident landmark blocks of the active
 * problems, captured as one HIP graph as the PCG iterations are, with HIP
 * events on the context stream around its second launch (the first warms
 * up); the autotuner times its candidates the same way; *bytes (may be NULL) receives
 * the algorithmic bytes of one product, 4 (18 k^2 + 9 k) per active landmark.
 * Overwrites only scratch (the product outputs). */
int32_t sqrtba_time_product(sqrtba_ctx* ctx, int32_t reps, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* SQRTBA_H */
