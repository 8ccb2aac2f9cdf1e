/*
 * sqrtba64.h -- C ABI of libsqrtba64.so: square-root bundle adjustment in
 * double precision (the FP64 variant of the method, Sec. 6: the paper runs its
 * solver in single and in double precision and compares the two).
 *
 * libsqrtba64.so is built from the same kernels and host code as libsqrtba.so
 * with every per-element quantity in FP64: camera and landmark state, pixels,
 * Jacobians, the stored landmark blocks (or per-observation records), the
 * Householder and Givens arithmetic, the preconditioner, the PCG vectors and
 * the back-substitution.  Per-problem sums are FP64 in both libraries.
 *
 * Every sqrtba64_X below has the contract of sqrtba_X in sqrtba.h (arguments,
 * layouts, ownership, state rules, status codes, options and report structs),
 * with two differences:
 *  - every array that is float in sqrtba.h is double here (state in and out,
 *    pixels, and the debug outputs), same shape and layout;
 *  - the learned preconditioner and its training (sqrtba_mlp_*,
 *    sqrtba_set_preconditioner, sqrtba_pcg_trace, sqrtba_trace_size,
 *    sqrtba_learned_stats, sqrtba_debug_features,
 *    sqrtba_debug_learned_precond) are FP32 only and not exported: the FP64
 *    library always uses the block-Jacobi preconditioner.
 * Device memory per element doubles, so the workspace of a problem is about
 * twice that of libsqrtba.so (sqrtba64_workspace_bytes reports it).
 * Contexts of the two libraries are distinct types and never interchangeable.
 */
#ifndef SQRTBA64_H
#define SQRTBA64_H

#include "sqrtba.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sqrtba64_ctx sqrtba64_ctx;

/* Lifetime and options: as sqrtba_version ... sqrtba_last_error.  The options struct is shared; the
 * FP64 context validates it the same way (SQRTBA_E_INVALID). */
int32_t sqrtba64_version(void);
void sqrtba64_default_options(sqrtba_options* opt);
int32_t sqrtba64_create(sqrtba64_ctx** out, const sqrtba_options* opt, void* hip_stream);
int32_t sqrtba64_set_options(sqrtba64_ctx* ctx, const sqrtba_options* opt);
void sqrtba64_destroy(sqrtba64_ctx* ctx);
const char* sqrtba64_last_error(const sqrtba64_ctx* ctx);

/* Problem definition (Sec. 4, Sec. 6.2 camera model): host arrays, copied during the call.
 * Cameras n_cams x 9 doubles (w, t, f, k1, k2), landmarks n_points x 3 doubles, pixels n_obs x 2
 * doubles; the same validation and bookkeeping as sqrtba_set_*. */
int32_t sqrtba64_set_problems(sqrtba64_ctx* ctx, int32_t n_problems, const int64_t* cam_off,
                              const int64_t* pt_off);
int32_t sqrtba64_set_cameras(sqrtba64_ctx* ctx, int64_t n_cams, const double* params);
int32_t sqrtba64_set_landmarks(sqrtba64_ctx* ctx, int64_t n_points, const double* xyz);
int32_t sqrtba64_set_observations(sqrtba64_ctx* ctx, int64_t n_obs, const int32_t* cam, const int32_t* pt,
                                  const double* uv);
/* device-pointer forms (sqrtba_set_*_device, sqrtba_get_*_device) */
int32_t sqrtba64_set_cameras_device(sqrtba64_ctx* ctx, int64_t n_cams, const double* params);
int32_t sqrtba64_set_landmarks_device(sqrtba64_ctx* ctx, int64_t n_points, const double* xyz);
int32_t sqrtba64_set_observations_device(sqrtba64_ctx* ctx, int64_t n_obs, const int32_t* cam, const int32_t* pt,
                                         const double* uv);

/* Device workspace: about twice the FP32 size (every element is 8 bytes); owned by the caller when
 * bound, otherwise allocated by the library on first use (SQRTBA_E_OOM when it does not fit). */
int32_t sqrtba64_workspace_bytes(const sqrtba64_ctx* ctx, uint64_t* bytes);
int32_t sqrtba64_bind_workspace(sqrtba64_ctx* ctx, void* device_ptr, uint64_t bytes);
int32_t sqrtba64_set_active(sqrtba64_ctx* ctx, const uint8_t* mask);

/* One Levenberg-Marquardt attempt, every step in FP64: linearize (Sec. 4.1), marginalize by QR
 * (Sec. 4.3, 5.2), damp (Sec. 5.3), PCG on the reduced camera system (Sec. 5.4, eq. cg_mult),
 * back-substitute (eq. backsub_nm), update and commit (Sec. 6.1); then the whole loop. Scalars per
 * problem ([P] arrays) as in sqrtba.h; the same state rules (SQRTBA_E_STATE out of order). */
int32_t sqrtba64_linearize(sqrtba64_ctx* ctx, double* cost);
int32_t sqrtba64_marginalize(sqrtba64_ctx* ctx);
int32_t sqrtba64_damp(sqrtba64_ctx* ctx, const double* lambda);
int32_t sqrtba64_solve(sqrtba64_ctx* ctx, int32_t* iters, double* rel_res, int32_t* pcg_status);
int32_t sqrtba64_back_substitute(sqrtba64_ctx* ctx, double* model_decrease);
int32_t sqrtba64_update(sqrtba64_ctx* ctx, double* new_cost);
int32_t sqrtba64_commit(sqrtba64_ctx* ctx, const uint8_t* accept);
int32_t sqrtba64_lm_solve(sqrtba64_ctx* ctx, sqrtba_lm_report* report);
int32_t sqrtba64_lm_solve_tracked(sqrtba64_ctx* ctx, const double* tol_cost, sqrtba_lm_report* report);
int32_t sqrtba64_get_lm_history(const sqrtba64_ctx* ctx, int32_t problem, sqrtba_lm_record* out,
                                int32_t capacity, int32_t* n_records);

/* State out: n_cams x 9 and n_points x 3 doubles, written before the call returns. */
int32_t sqrtba64_get_cameras(sqrtba64_ctx* ctx, double* params);
int32_t sqrtba64_get_landmarks(sqrtba64_ctx* ctx, double* xyz);
int32_t sqrtba64_get_cameras_device(sqrtba64_ctx* ctx, double* params);
int32_t sqrtba64_get_landmarks_device(sqrtba64_ctx* ctx, double* xyz);

/* Inspection exports used by the tests, with the layouts of sqrtba_debug_* in double. */
int32_t sqrtba64_debug_bookkeeping(const sqrtba64_ctx* ctx, int64_t* n_active, int64_t* obs_perm,
                                   int64_t* lm_off, uint8_t* lm_active, uint8_t* cam_active);
int32_t sqrtba64_debug_linearization(sqrtba64_ctx* ctx, double* r, double* Jp, double* Jl);
int32_t sqrtba64_debug_scales(sqrtba64_ctx* ctx, double* s_cam, double* s_pt);
int32_t sqrtba64_debug_rcs_matvec(sqrtba64_ctx* ctx, int32_t m, const double* v, double* out);
/* sqrtba_rcs_matvec_noalloc in double precision (device pointers, no allocation; the
 * FP64 library holds its own array of SQRTBA_NOALLOC_SCRATCH_BYTES per GPU). */
int32_t sqrtba64_rcs_matvec_noalloc(sqrtba64_ctx* ctx, const double* v, double* out);
int32_t sqrtba64_debug_rhs(sqrtba64_ctx* ctx, double* rhs);
int32_t sqrtba64_debug_precond(sqrtba64_ctx* ctx, double* minv);
int32_t sqrtba64_debug_block(sqrtba64_ctx* ctx, int64_t pt, int32_t* k, double* out, double* factors);
int32_t sqrtba64_debug_solution(sqrtba64_ctx* ctx, double* dxp_scaled, double* dxl);
int32_t sqrtba64_debug_set_pose_increment(sqrtba64_ctx* ctx, const double* dxp_scaled);

/* Stage timing, state snapshots, product launch shapes and product timing, as in sqrtba.h;
 * the FP64 product has its own autotuned shapes. */
int32_t sqrtba64_profile_enable(sqrtba64_ctx* ctx, int32_t on);
int32_t sqrtba64_profile_get(const sqrtba64_ctx* ctx, sqrtba_profile* out);
int32_t sqrtba64_save_state(sqrtba64_ctx* ctx);
int32_t sqrtba64_restore_state(sqrtba64_ctx* ctx);
int32_t sqrtba64_get_tuning(sqrtba64_ctx* ctx, sqrtba_tuning* out);
int32_t sqrtba64_set_tuning(sqrtba64_ctx* ctx, const sqrtba_tuning* shape);
int32_t sqrtba64_autotune(sqrtba64_ctx* ctx, int32_t reps, sqrtba_tuning* best, sqrtba_tuning_trial* trials,
                          int32_t max_trials, int32_t* n_trials);
int32_t sqrtba64_time_product(sqrtba64_ctx* ctx, int32_t reps, double* ms, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* SQRTBA64_H */
