// Internal interface between the host library (api.cpp) and the HIP kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sqrtba {

// Element type of the whole path: FP32 (square-root BA-32), or FP64 when built
// with SQRTBA_FP64 (square-root BA-64, the double-precision variant of Sec. 6).
// Per-problem sums are FP64 in both.
#ifdef SQRTBA_FP64
typedef double real;
typedef double2 real2;
typedef double3 real3;
typedef double4 real4;
__host__ __device__ inline real2 make_real2(real a, real b) { return make_double2(a, b); }
__host__ __device__ inline real3 make_real3(real a, real b, real c) { return make_double3(a, b, c); }
__host__ __device__ inline real4 make_real4(real a, real b, real c, real d) { return make_double4(a, b, c, d); }
#else
typedef float real;
typedef float2 real2;
typedef float3 real3;
typedef float4 real4;
__host__ __device__ inline real2 make_real2(real a, real b) { return make_float2(a, b); }
__host__ __device__ inline real3 make_real3(real a, real b, real c) { return make_float3(a, b, c); }
__host__ __device__ inline real4 make_real4(real a, real b, real c, real d) { return make_float4(a, b, c, d); }
#endif

// Landmark work is split into size classes by observation count k; each class
// maps one landmark to a "team" of lanes of a fixed size.  The classes are
// contiguous k ranges; landmarks are ordered by decreasing k so the largest
// blocks start first.  One definition serves host bucketing and device dispatch.
enum { NUM_CLASSES = 6 };
//                               class:  0   1   2   3    4    5
__host__ __device__ constexpr int class_kmax(int c) {
  return c == 0 ? 3 : c == 1 ? 7 : c == 2 ? 14 : c == 3 ? 28 : c == 4 ? 113 : 512;
}
__host__ __device__ constexpr int class_team(int c) {
  return c == 0 ? 8 : c == 1 ? 16 : c == 2 ? 32 : c == 3 ? 64 : 256;
}
__host__ __device__ constexpr int class_of_k(int k) {
  return k <= 3 ? 0 : k <= 7 ? 1 : k <= 14 ? 2 : k <= 28 ? 3 : k <= 113 ? 4 : k <= 512 ? 5 : -1;
}

// Small per-landmark record (elements): R1 upper (6), Q1^T r (3), damped R upper (6),
// damped Q1^T r (3), landmark column scales (3), lambda used (1), pad (2), and for
// implicit landmark blocks the damping part D = N^T N = lambda (R1 R1^T + lambda I)^-1
// of the landmark's projector (N the damping rows of the rotated unit columns; 6,
// upper triangle row by row, 4-element aligned), pad (2).
enum {
  LMD_R = 0, LMD_QR = 6, LMD_RH = 9, LMD_QRH = 15, LMD_SL = 18, LMD_LAM = 21, LMD_P = 24, LMD_STRIDE = 32
};

// Implicit landmark blocks: per observation a record of 7 real4 "planes" holding
// the unscaled pose Jacobian rows (2 x 9, row by row, planes 0..4), the
// observation's two rows of the thin QR factor Q1 (2 x 3, planes 4..5), and in
// plane 6 the residual (2) and 2 zeros; the camera index is in rec_cam.  Records are in
// slot order (slot_zoff[slot] + o for observation o of a slot) and plane-major:
// plane p of record i is real4 p * NO + i, so a team reading one plane of its
// landmark's observations, and consecutive teams of consecutive landmarks, read
// contiguous memory.
enum { REC_PLANES = 7 };

// Device view of the whole context.  All pointers are device pointers.
struct Dev {
  int32_t P;       // problems
  int32_t NC;      // cameras
  int32_t NL;      // landmarks
  int32_t NS;      // active landmarks (slots)
  int32_t NO;      // active observations
  // camera state: 16 elements per camera: R (row-major 9), t (3), f, k1, k2, pad
  real* cam;
  real* cam_new;
  real4* pts;      // x, y, z, 0
  real4* pts_new;
  // sorted active observations (landmark-major, camera ascending)
  int32_t* obs_cam;
  int32_t* obs_lm;
  real2* obs_uv;
  int32_t* cam_obs_off;  // NC + 1
  int32_t* cam_obs_idx;  // NO, sorted-observation positions per camera
  int32_t* cam_prob;     // NC
  int32_t* lm_prob;      // NL
  int32_t* prob_cam_off; // P + 1
  int32_t* prob_lm_off;  // P + 1
  // slots (active landmarks in processing order)
  int32_t* slot_lm;
  int32_t* slot_k;
  int32_t* slot_obs0;
  int32_t* slot_prob;
  int64_t* slot_boff;  // element offset of the B rows (2k x W) in poolB (32-element aligned)
  int64_t* slot_toff;  // element offset of the undamped top rows (3 x W) in poolT (32-element aligned)
  int32_t* slot_zoff;  // element offset of the landmark's W product outputs in obsbuf (4-element aligned);
                       // implicit blocks: index of the landmark's first record (outputs at 12 x record)
  int32_t* cam_zpos;   // NO: obsbuf offset of the outputs of each camera's observations (camera order)
  int32_t* lm_slot;    // NL, -1 when inactive
  // row-block product of the largest landmarks: one job per block of
  // Launch::huge_rows rows (x: slot, y: row block), partial outputs per block
  int2* qjob;     // class-5 QR row chunks: (slot, first row | end row << 16)
  int2* hjob;
  int64_t* hz_off;  // per slot with k >= 29 (a prefix of the slots): offset of its partials in zpart
  real* zpart;
  real* poolB;
  real* poolT;
  real* lmd;     // NS * LMD_STRIDE
  real* rhoB;    // 2 * NO: residual column of the B rows of each landmark
  real* s_cam;   // NC * 9
  real* cam_jtj; // NC * 54: per camera J^T J (45, upper triangle row by row) and J^T r (9) of the
                 // linearization, unscaled and robust-weighted (block-Jacobi of explicit blocks)
  // PCG vectors (9 NC each)
  real* vx;
  real* vr;
  real* vz;
  real* vzs;     // NC * 12: S z per camera, 9 elements and 3 zero pad (4-element aligned), kept by the
                  // PCG kernels for the products' gather (outside PCG: S of the vector to multiply)
  real* vp;
  real* vq;
  real* vb;      // right-hand side b~
  real* minv;    // NC * 81 inverse preconditioner blocks
  real* obsrec;  // implicit blocks: REC_PLANES * NO real4 per-observation records (else null)
  int32_t* rec_cam;  // implicit blocks: NO camera indices of the records (else null)
  int32_t implicit;  // 1: implicit landmark blocks or (with sc) the explicit Schur complement:
                     // per-observation records, no poolB / poolT / rhoB
  // explicit Schur complement in FP32 (landmark_blocks = 2; the comparator of the paper's
  // explicit solver).  Records hold J_p, the unscaled J_l and r; per landmark H_ll and b_l
  // (scaled) sit in the R / QR slots of lmd and (H_ll + lambda I)^-1 in the P slot.
  int32_t sc;
  int32_t sc_noff;       // off-diagonal camera-pair blocks (then NC diagonal blocks)
  real* scb;            // (sc_noff + NC) * 81 elements, full 9 x 9, unscaled pose coordinates
  int32_t* sc_coff;      // sc_noff + 1: contributions of each off-diagonal block (CSR)
  int4* sc_contrib;      // (record a, record b, slot, 0), a of the block's first camera
  int32_t* sc_rowoff;    // NC + 1: blocks of each camera's row of the reduced matrix (CSR)
  int2* sc_rowent;       // (block | transposed << 31, other camera)
  real* vy;             // 9 NC: the Schur-complement product of the last launch
  int32_t* done_host;    // P ints in coherent pinned host memory (device view): the done flags of
                         // the last convergence test, written by the PCG update kernel, read by the
                         // host between chunks of iterations without a copy
  int32_t* pcg_skip;     // 1 int: some problem is inactive or done in the running PCG solve (the
                         // products then test a landmark's problem before reading its data)
  real* obsbuf;  // NO * 54 elements: per-observation preconditioner terms (implicit blocks and the
                  // explicit Schur complement); the product outputs reuse it in per-landmark aligned
                  // regions (slot_zoff)
  real* ttop;    // explicit blocks: NO * 32 elements, per observation the damped top rows' 3 x 9
                 // camera entries (row-major), then q^ (3) and 2 zeros; written by the damping
  real* dxl;     // NL * 3, unscaled landmark increment
  double* cam_part;  // NC, per-camera partial sums
  double* cam_part2; // NC
  double* cam_part3; // NC
  double* lm_part;   // NL, per-landmark partial sums
  double* psum;      // P * sum_chunks: chunk sums of the per-problem sums
  int32_t sum_chunks;  // chunks of SUM_CHUNK values in the longest per-problem range (landmarks or cameras)
  // per-problem scalars
  double* lambda;
  double* rz_next;  // r.z of the last update, for alpha
  double* beta;
  double* rz;
  double* rr;
  double* rr0;
  int32_t* iters;
  int32_t* done;
  int32_t* pstatus;
  double* qmod;      // PCG quadratic model at the current iterate (forcing test)
  double* dqmod;     // its change in the last update
  double* pcost;
  double* ppred;
  uint8_t* active;
  int32_t all_active;  // 1: every problem is active (the per-landmark stages then skip the flag test)
  int32_t test_sep;    // 1: the PCG convergence test is its own kernel after each update (k_pcg_test)
  uint8_t* flag;     // generic per-problem mask (relinearize / accept)
  int32_t* chol_fail;  // count of preconditioner blocks that fell back to the diagonal
  float* feats;        // NC * 64 learned-preconditioner features of the last preconditioner build
  float* lfac;         // NC * 45 lower Cholesky factors of the damped blocks (packed rows)
  float* cam_stats;    // NC * 4: log(1 + #obs), log(1 + #covisible cameras), mean and max log k
  real* cam_snap;     // saved state (save/restore)
  real4* pts_snap;
  real pcg_tol;
  real pcg_eta;     // > 0: Nash-Sofer truncation of PCG
  real huber;       // Huber parameter in pixels (0: squared loss)
};

struct WorkClass {
  int first_slot;  // first slot of this class (slots of a class are contiguous)
  int slots;       // number of slots
};

// Smallest row block of the row-block product (sizes the job list and the
// partial outputs); the tuned block size is a multiple of it.
enum { HUGE_ROWS_MIN = 64 };
// Bytes of rotated rows per workgroup of the class-5 QR (explicit blocks).
enum { QR_CHUNK_BYTES = 2 << 20 };
// Smallest bucket edge of the row-block product (sizes its slot range).
enum { ROWS_MIN_K = 29 };
// Values per chunk of the per-problem sums (kernels.hip, k_prob_sum_chunks).
enum { SUM_CHUNK_VALUES = 16384 };

struct Launch {
  // launch shapes of the product (set by the autotuner or sqrtba_set_tuning)
  int n45;         // slots with k >= 29 (classes 5 and 4, a prefix of the slots)
  int rows_min_k;  // bucket edge: landmarks with k >= rows_min_k take the row-block kernel
  int rows_n;      // their number (a prefix of the slots)
  int hjobs;       // number of row-block jobs for huge_rows
  int huge_rows;   // rows per job (>= 2 * 512: one job per landmark)
  int huge_side;   // row-block jobs on the side stream, concurrent with the rest
  int large_sep;   // the rest of k >= 29 as its own launch (else inside the small-class launch)
  int mv_rbs;      // row-batch set of the small classes (0: 4 rows, 1: 8 rows)
  int persist;     // > 0: the small-class launch is persistent with this many workgroups
  int nt;          // non-temporal block loads: bit 0 the row-block and four-wavefront kernels, bit 1 classes 0..3
  int qjobs;       // row-chunk jobs of the class-5 QR (explicit blocks)
  hipStream_t stream;
  hipStream_t side;   // second stream for the largest landmarks (may be null)
  hipEvent_t fork, join;
  WorkClass wc[NUM_CLASSES];
};

// kernel launchers (kernels.hip); return hipSuccess or the launch error
hipError_t launch_cam_linearize(const Dev& d, const Launch& L, bool jac, bool use_new, const uint8_t* mask);
hipError_t launch_prob_sum(const Dev& d, const Launch& L, const double* vals, const int32_t* off, double* out,
                           const uint8_t* mask);
hipError_t launch_marginalize(const Dev& d, const Launch& L, const uint8_t* mask);
hipError_t launch_damp(const Dev& d, const Launch& L, const uint8_t* mask);
hipError_t launch_precond_rhs(const Dev& d, const Launch& L);
hipError_t launch_pcg_init(const Dev& d, const Launch& L);
hipError_t launch_pcg_iteration(const Dev& d, const Launch& L);
hipError_t launch_matvec(const Dev& d, const Launch& L);      // the PCG product (p folded in)
hipError_t launch_pcg_vector(const Dev& d, const Launch& L);  // q and update of one iteration
hipError_t launch_pcg_final(const Dev& d, const Launch& L);   // test of the last update of a solve
hipError_t launch_backsub(const Dev& d, const Launch& L);
hipError_t launch_update(const Dev& d, const Launch& L);
hipError_t launch_commit(const Dev& d, const Launch& L);
// test helpers
hipError_t launch_matvec_only(const Dev& d, const Launch& L, const real* v_scaled, real* out);

// Scratch of the no-allocation product (noalloc.hip): a static device array of
// this many bytes per device, holding the scaled input vector (12 elements per
// camera), the product's per-observation outputs and then its row-block
// partials, each part rounded up to 64 elements.
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
// Device address of the array on `device` (which must be current), looked up
// once per device and kept.
hipError_t noalloc_scratch(int device, void** out);
int64_t noalloc_out_elems(int64_t out_elems);
// Elements of the array one call uses (cameras, output and row-block partial elements).
int64_t noalloc_elems(int64_t n_cams, int64_t out_elems, int64_t partial_elems);
// launch_matvec_only with the product's scratch in the array at scratch_ptr.
hipError_t launch_matvec_noalloc(const Dev& d, const Launch& L, void* scratch_ptr, int64_t out_elems,
                                 const real* v, real* out);
hipError_t launch_matvec_timing(const Dev& d, const Launch& L);  // product of z over all active landmarks
// S z into vzs once, before timed launch_matvec_timing calls (which then read it)
hipError_t launch_prescale_z(const Dev& d, const Launch& L);
hipError_t launch_debug_linearization(const Dev& d, const Launch& L, real* r, real* Jp, real* Jl);

}  // namespace sqrtba
