// HIP kernels of the square-root bundle-adjustment hot path, written for
// gfx950 (CDNA4, 64-lane wavefronts).  The element type `real` is FP32, or FP64
// when built with SQRTBA_FP64 (the double-precision variant of the method);
// sums across cameras, landmarks and observations of one problem are
// accumulated in FP64 with fixed-shape trees, so every result is run-to-run
// deterministic.
//
// Landmark-centric kernels (marginalize, damp, preconditioner/RHS, matvec,
// back-substitution) give each landmark a team of 8, 16, 32, 64 or 256 lanes
// chosen by its observation count k (4 to 64 lanes in the per-observation
// forms).  A team of <= 64 lanes lives inside one wavefront and reduces with
// DPP row operations (no LDS, no barrier); a team of 256 lanes is a whole
// workgroup.  Per-camera sums are never formed with atomics: the landmark
// kernels write per-observation results and camera kernels sum them over each
// camera's observation list.
//
// The matrix algebra is the paper's: nullspace marginalization by QR of each
// landmark's J_l (Sec. 4.3, Householder variant of Sec. 5.2), landmark damping
// by six Givens rotations (Sec. 5.3), and CG on the reduced normal equations
// with the product (Q2^T J_p)^T (Q2^T J_p v) + lambda v (Sec. 5.4, eq. cg_mult).
// Beside the stored blocks: the same reduced system from per-observation
// records (implicit blocks, J_p^T (I - Q1 P Q1^T) J_p), the explicit FP32
// Schur complement of the paper's comparison solver (Sec. 4.2), and the Huber
// loss of the experiments applied by IRLS (Sec. 6.2).

#include <hip/hip_runtime.h>

#include "device.h"

namespace sqrtba {

namespace {

constexpr int WG = 256;

__device__ __forceinline__ int width_of(int k) { return (9 * k + 3) & ~3; }

// ---------------------------------------------------------------- reductions

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// A 64-bit value moves as its two 32-bit halves under the same lane pattern.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// All-reduce over aligned groups of TEAM lanes (4, 8, 16, 32 or 64).  Every lane
// of the group receives the bitwise-identical sum (each step adds a commutative
// pair).  All lanes of a group must be active together.
template <int TEAM>
__device__ __forceinline__ real team_sum(real v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (TEAM >= 8) v += dpp_mov<0x141>(v);  // row_half_mirror: pairs quads of a half row
  if constexpr (TEAM >= 16) v += dpp_mov<0x140>(v);  // row_mirror: pairs half rows
  if constexpr (TEAM >= 32) v += __shfl_xor(v, 16);  // pairs rows of 16 within 32 lanes
  if constexpr (TEAM >= 64) v += __shfl_xor(v, 32);
  return v;
}

// The value v of lane j of the caller's team (j < TEAM <= 64).
template <int TEAM>
__device__ __forceinline__ real team_lane(real v, int j) {
  static_assert(TEAM <= 64, "a team within one wavefront");
  return __shfl(v, j, TEAM);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ real wave_sum_f(real v) { return team_sum<64>(v); }

// Workgroup all-reduce of a float (256 lanes = 4 waves), deterministic.
__device__ __forceinline__ real block_sum(real v, real* red4) {
  v = wave_sum_f(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red4[w] = v;
  __syncthreads();
  return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}

template <int TEAM>
__device__ __forceinline__ real tsum(real v, real* red4) {
  if constexpr (TEAM <= 64)
    return team_sum<TEAM>(v);
  else
    return block_sum(v, red4);
}

// Visibility of LDS writes to the rest of the team.
template <int TEAM>
__device__ __forceinline__ void team_sync() {
  if constexpr (TEAM <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// ------------------------------------------------------------- camera model

struct Cam {
  real R[9];
  real t[3];
  real f, k1, k2;
};

__device__ __forceinline__ void load_cam(const real* __restrict__ cam, int c, Cam& C) {
  const real4* p = reinterpret_cast<const real4*>(cam + 16 * (size_t)c);
  real4 a = p[0], b = p[1], d = p[2], e = p[3];
  C.R[0] = a.x; C.R[1] = a.y; C.R[2] = a.z; C.R[3] = a.w;
  C.R[4] = b.x; C.R[5] = b.y; C.R[6] = b.z; C.R[7] = b.w;
  C.R[8] = d.x; C.t[0] = d.y; C.t[1] = d.z; C.t[2] = d.w;
  C.f = e.x; C.k1 = e.y; C.k2 = e.z;
}

// BAL projection: P = R X + t, p = -P_xy / P_z, pi = f (1 + k1 |p|^2 + k2 |p|^4) p,
// r = pi - uv.  With JAC, Jp (2x9) w.r.t. (left rotation increment, t, f, k1, k2)
// and Jl (2x3) w.r.t. X.
template <bool JAC>
__device__ __forceinline__ void project(const Cam& C, real X0, real X1, real X2, real u, real v,
                                        real r[2], real Jp[2][9], real Jl[2][3]) {
  const real RX0 = C.R[0] * X0 + C.R[1] * X1 + C.R[2] * X2;
  const real RX1 = C.R[3] * X0 + C.R[4] * X1 + C.R[5] * X2;
  const real RX2 = C.R[6] * X0 + C.R[7] * X1 + C.R[8] * X2;
  const real P0 = RX0 + C.t[0], P1 = RX1 + C.t[1], P2 = RX2 + C.t[2];
  const real iz = 1.0f / P2;
  const real p0 = -P0 * iz, p1 = -P1 * iz;
  const real n2 = p0 * p0 + p1 * p1;
  const real d = 1.0f + n2 * (C.k1 + C.k2 * n2);
  const real fd = C.f * d;
  r[0] = fd * p0 - u;
  r[1] = fd * p1 - v;
  if constexpr (JAC) {
    // dpi/dp = f (d I + g p p^T), g = 2 (k1 + 2 k2 |p|^2)
    const real fg = C.f * 2.0f * (C.k1 + 2.0f * C.k2 * n2);
    const real a00 = fd + fg * p0 * p0, a01 = fg * p0 * p1, a11 = fd + fg * p1 * p1;
    // dp/dP = [[-iz, 0, -p0 iz], [0, -iz, -p1 iz]]
    const real A00 = -a00 * iz, A01 = -a01 * iz, A02 = -(a00 * p0 + a01 * p1) * iz;
    const real A10 = -a01 * iz, A11 = -a11 * iz, A12 = -(a01 * p0 + a11 * p1) * iz;
    // rotation: dP/d(dw) = -[RX]_x = [[0, RX2, -RX1], [-RX2, 0, RX0], [RX1, -RX0, 0]]
    Jp[0][0] = -A01 * RX2 + A02 * RX1;
    Jp[0][1] = A00 * RX2 - A02 * RX0;
    Jp[0][2] = -A00 * RX1 + A01 * RX0;
    Jp[1][0] = -A11 * RX2 + A12 * RX1;
    Jp[1][1] = A10 * RX2 - A12 * RX0;
    Jp[1][2] = -A10 * RX1 + A11 * RX0;
    Jp[0][3] = A00; Jp[0][4] = A01; Jp[0][5] = A02;
    Jp[1][3] = A10; Jp[1][4] = A11; Jp[1][5] = A12;
    Jp[0][6] = d * p0;          Jp[1][6] = d * p1;
    Jp[0][7] = C.f * n2 * p0;   Jp[1][7] = C.f * n2 * p1;
    Jp[0][8] = C.f * n2 * n2 * p0; Jp[1][8] = C.f * n2 * n2 * p1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Jl[0][j] = A00 * C.R[j] + A01 * C.R[3 + j] + A02 * C.R[6 + j];
      Jl[1][j] = A10 * C.R[j] + A11 * C.R[3 + j] + A12 * C.R[6 + j];
    }
  }
}

// Huber loss by IRLS (delta > 0; delta = 0 is the squared loss): for the
// observation's s = |r|^2 the cost term rho(s) (s up to delta^2, then
// 2 delta sqrt(s) - delta^2) and the row weight sqrt(rho'(s)) =
// sqrt(min(1, delta / |r|)) that scales its residual and Jacobian rows.
__device__ __forceinline__ real robust_term(real s, real delta, real& sqrt_w) {
  if (delta <= 0.f || s <= delta * delta) {
    sqrt_w = 1.0f;
    return s;
  }
  const real n = sqrt(s);
  sqrt_w = sqrt(delta / n);
  return 2.0f * delta * n - delta * delta;
}

// ---------------------------------------------------- kernel (a): per camera

// One wavefront per camera: cost (FP64 sum of the FP32 per-observation terms,
// |r|^2 or the Huber rho) and, with JAC, the unit-norm scale of each of the
// camera's 9 (reweighted) Jacobian columns (1 / column norm; an empty column
// keeps scale 1).
template <bool JAC>
__global__ __launch_bounds__(64) void k_cam_linearize(Dev d, const real* __restrict__ cam,
                                                      const real4* __restrict__ pts, const uint8_t* mask) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  if (mask && !mask[d.cam_prob[c]]) return;
  Cam C;
  load_cam(cam, c, C);
  // JAC: the camera's (robust-weighted, unscaled) J^T J, upper triangle row by
  // row (45), and J^T r (9); its diagonal gives the column scales, and with
  // explicit blocks both feed the block-Jacobi blocks and the right-hand side
  constexpr int NJ = JAC ? 54 : 1;
  real jt[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) jt[j] = 0.f;
  double cost = 0.0;
  const int b = d.cam_obs_off[c], e = d.cam_obs_off[c + 1];
  for (int i = b + lane; i < e; i += 64) {
    const int o = d.cam_obs_idx[i];
    const real4 X = pts[d.obs_lm[o]];
    const real2 uv = d.obs_uv[o];
    real r[2], Jp[2][9], Jl[2][3];
    project<JAC>(C, X.x, X.y, X.z, uv.x, uv.y, r, Jp, Jl);
    real sw;
    cost += (double)robust_term(r[0] * r[0] + r[1] * r[1], d.huber, sw);
    if constexpr (JAC) {
      const real w = sw * sw;
      int q = 0;
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        jt[45 + a] += w * (Jp[0][a] * r[0] + Jp[1][a] * r[1]);
#pragma unroll
        for (int m = a; m < 9; ++m) jt[q++] += w * (Jp[0][a] * Jp[0][m] + Jp[1][a] * Jp[1][m]);
      }
    }
  }
  cost = wave_sum_d(cost);
  if constexpr (JAC) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) jt[j] = wave_sum_f(jt[j]);
    // lane j < 54 writes entry j; diagonal entry (a, a) sits at 9a - a(a-1)/2
    real v = jt[0];
#pragma unroll
    for (int j = 1; j < NJ; ++j) v = (lane == j) ? jt[j] : v;
    if (lane < NJ) d.cam_jtj[NJ * (size_t)c + lane] = v;
    if (lane < 9) {
      real n2 = jt[0];
#pragma unroll
      for (int a = 1; a < 9; ++a) n2 = (lane == a) ? jt[9 * a - a * (a - 1) / 2] : n2;
      d.s_cam[9 * c + lane] = n2 > 0.f ? 1.0f / sqrt(n2) : 1.0f;
    }
  }
  if (lane == 0) d.cam_part[c] = cost;
}

// Per-problem sums out[p] = sum of vals[off[p] .. off[p+1]) in two passes, so
// that a problem of a million landmarks does not leave the sum to one
// workgroup: chunk c of SUM_CHUNK values of problem p is summed by workgroup
// (p, c) into psum[p * chunks + c] (strided per thread, then the wavefront
// sums in a fixed order), and one wavefront per problem adds its chunks in a
// fixed tree.  The order depends only on the problem's own length, so a
// problem's sum has the same bits alone and in a batch.
constexpr int SUM_CHUNK = SUM_CHUNK_VALUES;
constexpr int SUM_THREADS = 256;

__global__ __launch_bounds__(SUM_THREADS) void k_prob_sum_chunks(const double* __restrict__ vals,
                                                                 const int32_t* __restrict__ off, double* psum,
                                                                 int chunks, const uint8_t* mask) {
  __shared__ double red[SUM_THREADS / 64];
  const int p = blockIdx.x / chunks, c = blockIdx.x % chunks;
  if (mask && !mask[p]) return;
  const int b = off[p] + c * SUM_CHUNK, e = min(off[p + 1], b + SUM_CHUNK);
  if (b >= e) return;  // uniform over the workgroup
  double s = 0.0;
#pragma unroll 8
  for (int i = b + (int)threadIdx.x; i < e; i += SUM_THREADS) s += vals[i];
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) psum[(size_t)p * chunks + c] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void k_prob_sum_final(const int32_t* __restrict__ off, const double* psum,
                                                       int chunks, double* out, const uint8_t* mask) {
  const int p = blockIdx.x;
  if (mask && !mask[p]) return;
  const int n = (off[p + 1] - off[p] + SUM_CHUNK - 1) / SUM_CHUNK;
  double s = 0.0;
  for (int c = (int)threadIdx.x; c < n; c += 64) s += psum[(size_t)p * chunks + c];
  s = wave_sum_d(s);
  if (threadIdx.x == 0) out[p] = s;
}

// Slot ranges of the size classes, in launch order (class 4, 3, 2, 1, 0):
// workgroup b of class j takes slots first[j] + b * (WG / team size) onwards
// (one slot per workgroup for class 4).  The slot of every team follows from
// blockIdx and these kernel arguments alone.
struct ClassGrid {
  int nblk[5];
  int first[5];
  int end[5];
};

// Runs f.run<TEAM, CLASS>(slot, lane, team) for the team of this thread in a
// launch over the classes 4..0 described by m (classes with nblk 0 are absent).
template <class F>
__device__ __forceinline__ void class_dispatch(const ClassGrid& m, const F& f) {
  int b = blockIdx.x;
  if (b < m.nblk[0]) { f.template run<256, 4>(m.first[0] + b, threadIdx.x, 0); return; }
  b -= m.nblk[0];
  if (b < m.nblk[1]) {
    const int t = threadIdx.x / 64, slot = m.first[1] + b * (WG / 64) + t;
    if (slot < m.end[1]) f.template run<64, 3>(slot, threadIdx.x % 64, t);
    return;
  }
  b -= m.nblk[1];
  if (b < m.nblk[2]) {
    const int t = threadIdx.x / 32, slot = m.first[2] + b * (WG / 32) + t;
    if (slot < m.end[2]) f.template run<32, 2>(slot, threadIdx.x % 32, t);
    return;
  }
  b -= m.nblk[2];
  if (b < m.nblk[3]) {
    const int t = threadIdx.x / 16, slot = m.first[3] + b * (WG / 16) + t;
    if (slot < m.end[3]) f.template run<16, 1>(slot, threadIdx.x % 16, t);
    return;
  }
  b -= m.nblk[3];
  const int t = threadIdx.x / 8, slot = m.first[4] + b * (WG / 8) + t;
  if (slot < m.end[4]) f.template run<8, 0>(slot, threadIdx.x % 8, t);
}

// ------------------------------------------- kernel (b): marginalize by QR

// Per landmark (team): linearize its k observations, scale the landmark columns
// to unit norm, factor J_l (2k x 3) = Q R with three Householder reflections
// H_j = I - tau_j v_j v_j^T, v_j = x + sign(x_j) |x| e_j (sign(0) = +1), and
// write Q^T [J_p | r].  Q^T = I - V T^T V^T (compact WY form, T upper
// triangular), so each output entry is the sparse J_p entry minus a rank-3
// correction: only O(k) values are combined, and the O(k^2) output is written
// once, coalesced, as float4 rows.
//   rows 0..2   -> undamped top rows [Q1^T J_p | R1 | Q1^T r] (poolT, lmd)
//   rows 3..2k-1 -> nullspace rows [Q2^T J_p | 0 | Q2^T r]    (poolB, rhoB)
//
// Each lane owns the observations o = lane, lane + TEAM, ... and their two rows
// (rows 2o, 2o + 1) from linearization through the reflections, in registers,
// so phases 1-3 need no LDS and no barrier besides the reductions; several
// independent sums are reduced together.  Only the reflectors V and the pose
// Jacobians go to LDS, for phase 4, where every lane needs every row.

// Sum over the team of N values per lane; every lane gets the same bits.  For
// TEAM <= 64 a DPP all-reduce; for a workgroup team, one barrier, with the
// wavefront partials in one of two LDS buffers (alternating, so a buffer is
// rewritten only after every thread has passed the barrier that follows the
// reads of its previous use).
template <int TEAM, int N>
__device__ __forceinline__ void team_sum_n(real (&v)[N], real* red, int& buf) {
  if constexpr (TEAM <= 64) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = team_sum<TEAM>(v[i]);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum_f(v[i]);
    real* r = red + buf * (4 * 8);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) r[8 * w + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = (r[i] + r[8 + i]) + (r[16 + i] + r[24 + i]);
    buf ^= 1;
  }
}

// Plane p of the implicit per-observation records (REC_PLANES planes of NO float4).
__device__ __forceinline__ real4* rec_plane(const Dev& d, int p) {
  return reinterpret_cast<real4*>(d.obsrec) + (size_t)p * d.NO;
}

// LDS floats per team: V (2k x 4) and the pose Jacobians (k x 18), rounded up
// to whole float4s so that every team's V is 16-byte aligned.
__host__ __device__ constexpr int marg_stride(int kmax) { return (26 * kmax + 3) & ~3; }
// LDS floats of the reductions of a workgroup team (two buffers of 4 x 8).
constexpr int MARG_RED = 64;

// Rows [row_lo, row_hi) of the rotated block are written (the whole block for
// 0, >= 2k); the landmark record and the residual rows are written by the
// chunk with row_lo = 0.
template <int TEAM, int KMAX, bool IMPLICIT>
__device__ __forceinline__ void marginalize_one(const Dev& d, int slot, int lane, real* lds, real* red,
                                                const uint8_t* mask, int row_lo = 0, int row_hi = 1 << 30) {
  constexpr int OPL = (KMAX + TEAM - 1) / TEAM;  // observations per lane
  const int prob = d.slot_prob[slot];
  if (mask && !mask[prob]) return;
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const int n = 2 * k;
  const int W = width_of(k);
  const int G = W >> 2;
  real4* V = reinterpret_cast<real4*>(lds);
  real* Jpc = lds + 8 * KMAX;
  const real4 X = d.pts[d.slot_lm[slot]];
  int buf = 0;

  // phase 1: residuals and Jacobians of the lane's observations
  real3 A[2 * OPL];   // rows 2o, 2o+1 of J_l (scaled below), o = lane + TEAM m
  real rr[2 * OPL];
  real cl[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    A[2 * m] = A[2 * m + 1] = make_real3(0.f, 0.f, 0.f);
    rr[2 * m] = rr[2 * m + 1] = 0.f;
    if (o < k) {
      Cam C;
      load_cam(d.cam, d.obs_cam[obs0 + o], C);
      const real2 uv = d.obs_uv[obs0 + o];
      real r[2], Jp[2][9], Jl[2][3];
      project<true>(C, X.x, X.y, X.z, uv.x, uv.y, r, Jp, Jl);
      real sw;
      (void)robust_term(r[0] * r[0] + r[1] * r[1], d.huber, sw);
      if (sw != 1.0f) {  // Huber IRLS: the observation's rows scaled by sqrt(w)
        r[0] *= sw;
        r[1] *= sw;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          Jp[0][j] *= sw;
          Jp[1][j] *= sw;
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Jl[0][j] *= sw;
          Jl[1][j] *= sw;
        }
      }
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        Jpc[18 * o + j] = Jp[0][j];
        Jpc[18 * o + 9 + j] = Jp[1][j];
      }
      A[2 * m] = make_real3(Jl[0][0], Jl[0][1], Jl[0][2]);
      A[2 * m + 1] = make_real3(Jl[1][0], Jl[1][1], Jl[1][2]);
      rr[2 * m] = r[0];
      rr[2 * m + 1] = r[1];
      cl[0] += Jl[0][0] * Jl[0][0] + Jl[1][0] * Jl[1][0];
      cl[1] += Jl[0][1] * Jl[0][1] + Jl[1][1] * Jl[1][1];
      cl[2] += Jl[0][2] * Jl[0][2] + Jl[1][2] * Jl[1][2];
    }
  }
  team_sum_n<TEAM, 3>(cl, red, buf);
  const real sl0 = cl[0] > 0.f ? 1.0f / sqrt(cl[0]) : 1.0f;
  const real sl1 = cl[1] > 0.f ? 1.0f / sqrt(cl[1]) : 1.0f;
  const real sl2 = cl[2] > 0.f ? 1.0f / sqrt(cl[2]) : 1.0f;
#pragma unroll
  for (int i = 0; i < 2 * OPL; ++i) {
    A[i].x *= sl0;
    A[i].y *= sl1;
    A[i].z *= sl2;
  }
  auto row_of = [&](int i) { return 2 * (lane + TEAM * (i >> 1)) + (i & 1); };  // own row i -> block row
  auto comp = [](const real3& a, int j) { return j == 0 ? a.x : (j == 1 ? a.y : a.z); };

  // phase 2: three Householder reflections on the scaled J_l
  real3 Vr[2 * OPL];
#pragma unroll
  for (int i = 0; i < 2 * OPL; ++i) Vr[i] = make_real3(0.f, 0.f, 0.f);
  real tau[3], alph[3], nrms[3], Rrow[3][3];  // Rrow: row j of R1 as seen by its owner
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    // |x|^2 over rows >= j and x_j itself (contributed by the owner of row j)
    real sx[2] = {0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 2 * OPL; ++i) {
      const int gi = row_of(i);
      const real x = comp(A[i], j);
      if (gi < n && gi >= j) sx[0] += x * x;
      if (gi == j) sx[1] = x;
    }
    team_sum_n<TEAM, 2>(sx, red, buf);
    const real nrm = sqrt(sx[0]), xj = sx[1];
    real alpha = 0.f, vj = 0.f, tj = 0.f;
    if (nrm > 0.f) {
      // v = x + sign(x_j) |x| e_j, so v^T v = 2 |x| (|x| + |x_j|) exactly: tau = 2 / v^T v
      // without the cancellation of |x|^2 - x_j^2 when x_j dominates the column
      alpha = xj >= 0.f ? -nrm : nrm;
      vj = xj - alpha;
      tj = 1.0f / (nrm * (nrm + fabs(xj)));
    }
    tau[j] = tj;
    alph[j] = alpha;
    nrms[j] = nrm;
    // reflector j on the lane's rows, and w_m = v^T a_m for the columns m > j
    real wv[2] = {0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 2 * OPL; ++i) {
      const int gi = row_of(i);
      const real x = comp(A[i], j);
      const real vi = (tj == 0.f || gi < j || gi >= n) ? 0.f : (gi == j ? vj : x);
      if (j == 0) Vr[i].x = vi; else if (j == 1) Vr[i].y = vi; else Vr[i].z = vi;
      if (j == 0) { wv[0] += vi * A[i].y; wv[1] += vi * A[i].z; }
      else if (j == 1) { wv[0] += vi * A[i].z; }
    }
    if (j == 0) {
      team_sum_n<TEAM, 2>(wv, red, buf);
    } else if (j == 1) {
      real w1[1] = {wv[0]};
      team_sum_n<TEAM, 1>(w1, red, buf);
      wv[0] = w1[0];
    }
    // apply H_j to the remaining columns m > j of the lane's rows
#pragma unroll
    for (int i = 0; i < 2 * OPL; ++i) {
      const real vi = comp(Vr[i], j);
      if (j == 0) { A[i].y -= tj * vi * wv[0]; A[i].z -= tj * vi * wv[1]; }
      else if (j == 1) { A[i].z -= tj * vi * wv[0]; }
    }
    // the owner of row j keeps it (entries of R1 right of the diagonal)
#pragma unroll
    for (int i = 0; i < 2 * OPL; ++i)
      if (row_of(i) == j) { Rrow[j][0] = A[i].x; Rrow[j][1] = A[i].y; Rrow[j][2] = A[i].z; }
  }

  // phase 3: T of the compact WY form (LAPACK larft, forward columnwise) and
  // V^T r, reduced together
  real dv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 2 * OPL; ++i) {
    const real3 vv = Vr[i];
    const real ri = rr[i];
    dv[0] += vv.x * vv.y; dv[1] += vv.x * vv.z; dv[2] += vv.y * vv.z;
    dv[3] += vv.x * ri; dv[4] += vv.y * ri; dv[5] += vv.z * ri;
  }
  team_sum_n<TEAM, 6>(dv, red, buf);
  const real d01 = dv[0], d02 = dv[1], d12 = dv[2], wr0 = dv[3], wr1 = dv[4], wr2 = dv[5];
  const real T00 = tau[0], T11 = tau[1], T22 = tau[2];
  const real T01 = -tau[1] * T00 * d01;
  const real T02 = -tau[2] * (T00 * d02 + T01 * d12);
  const real T12 = -tau[2] * (T11 * d12);
  // residual column: Q^T r = r - V (T^T (V^T r))
  const real mr0 = T00 * wr0;
  const real mr1 = T01 * wr0 + T11 * wr1;
  const real mr2 = T02 * wr0 + T12 * wr1 + T22 * wr2;
  real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const bool head = row_lo == 0;  // this chunk writes the landmark record
#pragma unroll
  for (int i = 0; i < 2 * OPL; ++i) {
    const int gi = row_of(i);
    if (gi < n) {
      const real3 vv = Vr[i];
      const real val = rr[i] - (vv.x * mr0 + vv.y * mr1 + vv.z * mr2);
      if (head) {
        if (gi < 3) lmd[LMD_QR + gi] = val;
        else if (!IMPLICIT) d.rhoB[2 * (size_t)obs0 + (gi - 3)] = val;
      }
      V[gi] = make_real4(vv.x, vv.y, vv.z, 0.f);
    }
    if (!head) continue;
    // R1: the diagonal is alpha_j (or the untouched entry when |x| = 0), the
    // rest of row j comes from its owner
    if (gi == 0) {
      lmd[LMD_R + 0] = nrms[0] > 0.f ? alph[0] : Rrow[0][0];
      lmd[LMD_R + 1] = Rrow[0][1];
      lmd[LMD_R + 2] = Rrow[0][2];
    } else if (gi == 1) {
      lmd[LMD_R + 3] = nrms[1] > 0.f ? alph[1] : Rrow[1][1];
      lmd[LMD_R + 4] = Rrow[1][2];
    } else if (gi == 2) {
      lmd[LMD_R + 5] = nrms[2] > 0.f ? alph[2] : Rrow[2][2];
    }
  }
  if (lane == 0 && head) {
    lmd[LMD_SL + 0] = sl0; lmd[LMD_SL + 1] = sl1; lmd[LMD_SL + 2] = sl2;
  }
  team_sync<TEAM>();  // V and the pose Jacobians of every row, for phase 4

  if constexpr (IMPLICIT) {
    // phase 4 (implicit blocks): per observation its record: the pose Jacobian
    // rows, its two rows of the thin factor Q1 = Q[:, 0:3] = E - V T V3^T (V3 the
    // top three rows of V, lower triangular) and its residual
    real K[3][3];  // K = T V3^T
    {
      const real4 v0 = V[0], v1 = V[1], v2 = V[2];
      const real v3[3][3] = {{v0.x, v0.y, v0.z}, {v1.x, v1.y, v1.z}, {v2.x, v2.y, v2.z}};
      const real T[3][3] = {{T00, T01, T02}, {0.f, T11, T12}, {0.f, 0.f, T22}};
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int j = 0; j < 3; ++j) K[m][j] = T[m][0] * v3[j][0] + T[m][1] * v3[j][1] + T[m][2] * v3[j][2];
    }
#pragma unroll
    for (int m = 0; m < OPL; ++m) {
      const int o = lane + TEAM * m;
      if (o < k) {
        real q[2][3];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const real3 vv = Vr[2 * m + h];
          const int gi = 2 * o + h;
#pragma unroll
          for (int j = 0; j < 3; ++j)
            q[h][j] = (gi == j ? 1.f : 0.f) - (vv.x * K[0][j] + vv.y * K[1][j] + vv.z * K[2][j]);
        }
        const real* J = Jpc + 18 * o;
        real4* rec = rec_plane(d, 0) + d.slot_zoff[slot] + o;
        const size_t P = (size_t)d.NO;
        rec[0] = make_real4(J[0], J[1], J[2], J[3]);
        rec[P] = make_real4(J[4], J[5], J[6], J[7]);
        rec[2 * P] = make_real4(J[8], J[9], J[10], J[11]);
        rec[3 * P] = make_real4(J[12], J[13], J[14], J[15]);
        rec[4 * P] = make_real4(J[16], J[17], q[0][0], q[0][1]);
        rec[5 * P] = make_real4(q[0][2], q[1][0], q[1][1], q[1][2]);
        rec[6 * P] = make_real4(rr[2 * m], rr[2 * m + 1], 0.f, 0.f);
      }
    }
    return;
  }

  // phase 4: pose columns, Q^T J_p = J_p - V M with M = T^T (V^T J_p).  Lane
  // g-groups are g = lane + TEAM jg; for a workgroup team the rows are the
  // outer loop, so every output row (up to 18 KB) is written whole, in order.
  // A workgroup team with one column group per lane (k <= 113: G <= 255)
  // would leave the lanes past G idle through the row loop; it takes
  // rstep = 256 / GP rows at a time instead (GP: G rounded up to whole
  // wavefronts), lane t writing column group t % GP of row i + t / GP.
  real* outT = d.poolT + d.slot_toff[slot];
  real* outB = d.poolB + d.slot_boff[slot];
  constexpr int NG = (((9 * KMAX + 3) / 4) + TEAM - 1) / TEAM;  // column groups per lane
  int glane = lane, rsub = 0, rstep = 1;
  if constexpr (TEAM == 256 && NG == 1) {
    const int GP = (G + 63) & ~63;  // 64 .. 256
    rstep = 256 / GP;
    glane = lane % GP;
    rsub = lane / GP;  // >= rstep: a lane with no row (256 not a multiple of GP)
  }
  real M0[NG][4], M1[NG][4], M2[NG][4], j0[NG][4], j1[NG][4];
  int row0[NG][4];
#pragma unroll
  for (int jg = 0; jg < NG; ++jg) {
    const int g = glane + TEAM * jg;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * g + q;
      M0[jg][q] = M1[jg][q] = M2[jg][q] = j0[jg][q] = j1[jg][q] = 0.f;
      row0[jg][q] = -4;
      if (g < G && c < 9 * k) {
        const int o = (unsigned)c / 9u;
        const int m = c - 9 * o;
        const real a0 = Jpc[18 * o + m], a1 = Jpc[18 * o + 9 + m];
        const real4 va = V[2 * o], vb = V[2 * o + 1];
        const real W0 = va.x * a0 + vb.x * a1;
        const real W1 = va.y * a0 + vb.y * a1;
        const real W2 = va.z * a0 + vb.z * a1;
        M0[jg][q] = T00 * W0;
        M1[jg][q] = T01 * W0 + T11 * W1;
        M2[jg][q] = T02 * W0 + T12 * W1 + T22 * W2;
        j0[jg][q] = a0;
        j1[jg][q] = a1;
        row0[jg][q] = 2 * o;
      }
    }
  }
  const int i_end = row_hi < n ? row_hi : n;
  for (int i = row_lo + rsub; i < i_end && rsub < rstep; i += rstep) {
    const real4 vv = V[i];
    real4* row = reinterpret_cast<real4*>(i < 3 ? outT + (size_t)i * W : outB + (size_t)(i - 3) * W);
#pragma unroll
    for (int jg = 0; jg < NG; ++jg) {
      const int g = glane + TEAM * jg;
      if (g < G) {
        real out[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const real base = (i == row0[jg][q]) ? j0[jg][q] : ((i == row0[jg][q] + 1) ? j1[jg][q] : 0.f);
          out[q] = base - (vv.x * M0[jg][q] + vv.y * M1[jg][q] + vv.z * M2[jg][q]);
        }
        row[g] = make_real4(out[0], out[1], out[2], out[3]);
      }
    }
  }
}

// ---------------------------------------------------- landmark damping

// The six Givens rotations that fold sqrt(lambda) I (three rows appended
// below R1) into the upper triangle: for damping row e = 0, 1, 2 and pivot
// row j = e..2, rotate (top row j, damping row e) so that entry (e, j) of the
// damping rows vanishes.  c = a / rho, s = b / rho with rho = hypot(a, b) of
// the pivot entry a and the entry b to remove; rho = 0 gives the identity.
// On return Rh holds the damped upper triangle, qrh the damped Q1^T r and
// dr the residuals of the three rotated damping rows.
struct Givens6 {
  real c[6], s[6];
};

__device__ __forceinline__ void damping_rotations(const real* lmd, real sqlam, Givens6& G, real Rh[3][3],
                                                  real qrh[3], real dr[3]) {
  real t[3][4];  // top rows: 3 landmark columns + residual
  t[0][0] = lmd[LMD_R + 0]; t[0][1] = lmd[LMD_R + 1]; t[0][2] = lmd[LMD_R + 2]; t[0][3] = lmd[LMD_QR + 0];
  t[1][0] = 0.f;            t[1][1] = lmd[LMD_R + 3]; t[1][2] = lmd[LMD_R + 4]; t[1][3] = lmd[LMD_QR + 1];
  t[2][0] = 0.f;            t[2][1] = 0.f;            t[2][2] = lmd[LMD_R + 5]; t[2][3] = lmd[LMD_QR + 2];
  int idx = 0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    real dd[4] = {0.f, 0.f, 0.f, 0.f};
    dd[e] = sqlam;
#pragma unroll
    for (int j = e; j < 3; ++j) {
      const real a = t[j][j], b = dd[j];
      const real rho = hypot(a, b);
      real c = 1.f, s = 0.f;
      if (rho > 0.f) { c = a / rho; s = b / rho; }
      G.c[idx] = c; G.s[idx] = s; ++idx;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const real tm = t[j][m], dm = dd[m];
        t[j][m] = c * tm + s * dm;
        dd[m] = -s * tm + c * dm;
      }
      dd[j] = 0.f;  // exactly eliminated
    }
    dr[e] = dd[3];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Rh[j][0] = t[j][0]; Rh[j][1] = t[j][1]; Rh[j][2] = t[j][2];
    qrh[j] = t[j][3];
  }
  Rh[1][0] = 0.f; Rh[2][0] = 0.f; Rh[2][1] = 0.f;
}

// Apply the same rotation sequence to one column: top rows t[3] (in: undamped,
// out: damped) and damping rows dd[3] (in: 0, out: the three new B rows).
__device__ __forceinline__ void rotate_column(const Givens6& G, real t[3], real dd[3]) {
  int idx = 0;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    dd[e] = 0.f;
#pragma unroll
    for (int j = e; j < 3; ++j) {
      const real c = G.c[idx], s = G.s[idx];
      ++idx;
      const real tm = t[j], dm = dd[e];
      t[j] = c * tm + s * dm;
      dd[e] = -s * tm + c * dm;
    }
  }
}

// Damping of every landmark block from its stored undamped top rows (so a new
// lambda never needs a new QR): writes the three damping rows of B, their
// residuals, and the damped R and Q1^T r into the landmark record; the same
// rotations give the damped top rows, whose camera entries go to the
// per-observation records of the block-Jacobi stage (ttop).
// Observations per chunk of the per-observation records (a multiple of 4, so
// that every chunk starts on a column group), and LDS floats per team.
__host__ __device__ constexpr int damp_chunk(int team) { return team >= 256 ? 64 : (team >= 16 ? team / 4 : 4); }
__host__ __device__ constexpr int damp_lds(int team) { return 3 * 9 * damp_chunk(team); }
constexpr int DAMP_LDS = (WG / 8) * damp_lds(8);  // the largest over the team sizes
static_assert(DAMP_LDS >= (WG / 16) * damp_lds(16) && DAMP_LDS >= (WG / 32) * damp_lds(32) &&
              DAMP_LDS >= (WG / 64) * damp_lds(64) && DAMP_LDS >= damp_lds(256), "LDS of the damping");

template <int TEAM>
__device__ __forceinline__ void damp_one(const Dev& d, int slot, int lane, const uint8_t* mask, real* lds) {
  const int prob = d.slot_prob[slot];
  if (mask && !mask[prob]) return;
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const int W = width_of(k);
  const int G = W >> 2;
  real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real lam = (real)d.lambda[prob];
  Givens6 Gv;
  real Rh[3][3], qrh[3], dr[3];
  damping_rotations(lmd, sqrt(lam), Gv, Rh, qrh, dr);
  if (lane == 0) {
    lmd[LMD_RH + 0] = Rh[0][0]; lmd[LMD_RH + 1] = Rh[0][1]; lmd[LMD_RH + 2] = Rh[0][2];
    lmd[LMD_RH + 3] = Rh[1][1]; lmd[LMD_RH + 4] = Rh[1][2]; lmd[LMD_RH + 5] = Rh[2][2];
    lmd[LMD_QRH + 0] = qrh[0]; lmd[LMD_QRH + 1] = qrh[1]; lmd[LMD_QRH + 2] = qrh[2];
    lmd[LMD_LAM] = lam;
  }
  if (lane < 3) d.rhoB[2 * (size_t)obs0 + 2 * k - 3 + lane] = dr[lane];
  const real4* T = reinterpret_cast<const real4*>(d.poolT + d.slot_toff[slot]);
  real4* B = reinterpret_cast<real4*>(d.poolB + d.slot_boff[slot] + (size_t)(2 * k - 3) * W);
  // the damped top rows of a chunk of CH observations go to LDS (3 rows of 9 CH
  // columns), from which the chunk's records leave as whole float4s
  constexpr int CH = damp_chunk(TEAM), CW = 9 * CH;
  real4* tt = reinterpret_cast<real4*>(d.ttop + (size_t)obs0 * 32);  // the landmark's k records
  for (int j0 = 0; j0 < k; j0 += CH) {
    const int nj = min(CH, k - j0);
    const int g0 = (9 * j0) >> 2, g1 = min(G, (9 * (j0 + nj) + 3) >> 2);
    for (int gg = lane; gg < g1 - g0; gg += TEAM) {
      const int g = g0 + gg;
      const real4 t0 = T[g], t1 = T[G + g], t2 = T[2 * G + g];
      real a[3], b[3];
      real4 o0, o1, o2, h0, h1, h2;  // damping rows, damped top rows
      a[0] = t0.x; a[1] = t1.x; a[2] = t2.x; rotate_column(Gv, a, b); o0.x = b[0]; o1.x = b[1]; o2.x = b[2];
      h0.x = a[0]; h1.x = a[1]; h2.x = a[2];
      a[0] = t0.y; a[1] = t1.y; a[2] = t2.y; rotate_column(Gv, a, b); o0.y = b[0]; o1.y = b[1]; o2.y = b[2];
      h0.y = a[0]; h1.y = a[1]; h2.y = a[2];
      a[0] = t0.z; a[1] = t1.z; a[2] = t2.z; rotate_column(Gv, a, b); o0.z = b[0]; o1.z = b[1]; o2.z = b[2];
      h0.z = a[0]; h1.z = a[1]; h2.z = a[2];
      a[0] = t0.w; a[1] = t1.w; a[2] = t2.w; rotate_column(Gv, a, b); o0.w = b[0]; o1.w = b[1]; o2.w = b[2];
      h0.w = a[0]; h1.w = a[1]; h2.w = a[2];
      B[g] = o0;
      B[G + g] = o1;
      B[2 * G + g] = o2;
      if (4 * gg < CW) {  // the chunk's last group may run past 9 CH columns (padding)
        reinterpret_cast<real4*>(lds)[gg] = h0;
        reinterpret_cast<real4*>(lds + CW)[gg] = h1;
        reinterpret_cast<real4*>(lds + 2 * CW)[gg] = h2;
      }
    }
    team_sync<TEAM>();
    for (int p = lane; p < 8 * nj; p += TEAM) {  // float4 q of record jj
      const int jj = p >> 3, q = p & 7;
      real v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * q + c;
        const int i = e / 9, a = e - 9 * i;
        v[c] = e < 27 ? lds[i * CW + 9 * jj + a] : (e < 30 ? qrh[e - 27] : 0.f);
      }
      tt[8 * (j0 + jj) + q] = make_real4(v[0], v[1], v[2], v[3]);
    }
    team_sync<TEAM>();
  }
}

// ------------------------------------- block-Jacobi blocks and right-hand side

// The camera blocks of B^T B and B^T rho_B follow from the camera's own
// Jacobian rows and each landmark's three damped top rows: the QR and the
// damping rotations are orthogonal and leave the column Gram of [J_p | r]
// (with the three zero rows of the damping system) unchanged, so for
// observation j of a landmark, with its camera slab of 9 columns,
//   B_j^T B_j   = J_j^T J_j - T^_j^T T^_j,
//   B_j^T rho_B = J_j^T r_j - T^_j^T q^,
// T^ the damped top rows (rotated from the stored undamped rows) and q^ the
// damped Q1^T r.  The camera sums of J_j^T J_j and J_j^T r_j come from the
// linearization (cam_jtj); the damping, which rotates the top rows anyway,
// writes each observation's T^_j (3 x 9) and q^ to its 32-element record
// (ttop), and k_precond_cam forms T^_j^T T^_j (45 upper entries) and
// T^_j^T q^ (9) per observation and subtracts their sums.  A landmark costs
// its 3 top rows instead of its 2k B rows, read once by the damping.  The
// subtraction is of quantities of the same order (B keeps (2k - 3) / 2k of a
// slab's squared norm on average); per camera the FP32 blocks agree with the
// direct sum over the B rows to the same 3e-7.

// The 54 terms of one observation slab from its three damped top rows (row i
// at rows[i W], 9 entries).
__device__ __forceinline__ void top_gram(const real* __restrict__ rows, int W, const real (&qh)[3], real (&g)[54]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    real b[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) b[e] = rows[i * W + e];
    int e = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      g[45 + a] += b[a] * qh[i];
#pragma unroll
      for (int c = a; c < 9; ++c) g[e++] += b[a] * b[c];
    }
  }
}

// Per camera (one wavefront): sum the per-observation blocks (explicit
// blocks: subtract them from the camera's J^T J and J^T r), scale, add
// lambda I, Cholesky-factor and invert the 9x9 block (a non-positive pivot
// falls back to the inverse diagonal and is counted), and form b~ = S g.
__global__ __launch_bounds__(64) void k_precond_cam(Dev d) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int prob = d.cam_prob[c];
  if (!d.active[prob]) return;
  real acc[54];
#pragma unroll
  for (int e = 0; e < 54; ++e) acc[e] = 0.f;
  const int b = d.cam_obs_off[c], e1 = d.cam_obs_off[c + 1];
  if (!d.implicit) {  // explicit blocks: the top-row terms from the damping's records
    for (int i = b + lane; i < e1; i += 64) {
      const real4* rec = reinterpret_cast<const real4*>(d.ttop + (size_t)d.cam_obs_idx[i] * 32);
      real t[32];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const real4 v = rec[q];
        t[4 * q] = v.x; t[4 * q + 1] = v.y; t[4 * q + 2] = v.z; t[4 * q + 3] = v.w;
      }
      const real qh[3] = {t[27], t[28], t[29]};
      real g[54];
#pragma unroll
      for (int e = 0; e < 54; ++e) g[e] = 0.f;
      top_gram(t, 9, qh, g);
#pragma unroll
      for (int e = 0; e < 54; ++e) acc[e] += g[e];
    }
  } else {
    for (int i = b + lane; i < e1; i += 64) {
      const real* src = d.obsbuf + (size_t)d.cam_obs_idx[i] * 54;
#pragma unroll
      for (int e = 0; e < 54; ++e) acc[e] += src[e];
    }
  }
#pragma unroll
  for (int e = 0; e < 54; ++e) acc[e] = wave_sum_f(acc[e]);
  if (lane != 0) return;
  if (!d.implicit) {  // explicit blocks: the camera's J^T J and J^T r less the top-row terms
    const real* jt = d.cam_jtj + 54 * (size_t)c;
#pragma unroll
    for (int e = 0; e < 54; ++e) acc[e] = jt[e] - acc[e];
  }
  real s[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) s[a] = d.s_cam[9 * c + a];
  const real lam = (real)d.lambda[prob];
  real P[9][9];
  int e = 0;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
#pragma unroll
    for (int q = a; q < 9; ++q) {
      const real v = s[a] * acc[e++] * s[q];
      P[a][q] = v;
      P[q][a] = v;
    }
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    P[a][a] += lam;
    d.vb[9 * c + a] = s[a] * acc[45 + a];
  }
  // Cholesky P = L L^T (lower, in place)
  real L[9][9];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    real dj = P[j][j];
#pragma unroll
    for (int q = 0; q < j; ++q) dj -= L[j][q] * L[j][q];
    if (!(dj > 0.f)) { ok = false; dj = 1.f; }
    const real ljj = sqrt(dj);
    L[j][j] = ljj;
    const real il = 1.0f / ljj;
#pragma unroll
    for (int i = j + 1; i < 9; ++i) {
      real v = P[i][j];
#pragma unroll
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      L[i][j] = v * il;
    }
#pragma unroll
    for (int i = 0; i < j; ++i) L[i][j] = 0.f;
  }
  real* mi = d.minv + 81 * (size_t)c;
  // features of the block for the learned preconditioner, and its Cholesky
  // factor (a failed factorization is replaced by the square root of the diagonal)
  {
    float* f = d.feats + 64 * (size_t)c;
    float* lf = d.lfac + 45 * (size_t)c;
    real tr = 0.f;
    int e2 = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      f[a] = logf(P[a][a]);
      f[45 + a] = logf(lam / P[a][a]);
      tr += P[a][a];
#pragma unroll
      for (int q = a + 1; q < 9; ++q) f[9 + e2++] = P[a][q] * rsqrtf(P[a][a] * P[q][q]);
    }
    f[54] = logf(lam);
#pragma unroll
    for (int a = 0; a < 4; ++a) f[55 + a] = d.cam_stats[4 * (size_t)c + a];
    f[59] = logf(tr / 9.f);
    f[60] = f[61] = f[62] = f[63] = 0.f;
    int e3 = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int q = 0; q <= a; ++q) lf[e3++] = ok ? L[a][q] : (a == q ? sqrt(P[a][a]) : 0.f);
  }
  if (!ok) {
    atomicAdd(d.chol_fail, 1);
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int q = 0; q < 9; ++q) mi[9 * a + q] = (a == q) ? 1.0f / P[a][a] : 0.f;
    return;
  }
  // inverse of L (lower), then M^-1 = L^-T L^-1
  real Li[9][9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
#pragma unroll
    for (int i = 0; i < 9; ++i) Li[i][j] = 0.f;
    Li[j][j] = 1.0f / L[j][j];
#pragma unroll
    for (int i = j + 1; i < 9; ++i) {
      real v = 0.f;
#pragma unroll
      for (int q = j; q < i; ++q) v -= L[i][q] * Li[q][j];
      Li[i][j] = v / L[i][i];
    }
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      real v = 0.f;
#pragma unroll
      for (int i = (a > q ? a : q); i < 9; ++i) v += Li[i][a] * Li[i][q];
      mi[9 * a + q] = v;
    }
  }
}

// ----------------------------------------------------- kernel (c): matvec

// Gather of the landmark's slice of the scaled direction vector for the 4
// columns of column group g: p'[c] = (S v)[cam, m], read from vs, which holds
// S v with 12 elements per camera (9 values and 3 pad, as vzs).  Columns past
// 9k read a valid entry and give 0 (no conditional loads).
__device__ __forceinline__ real4 gather_cols(const Dev& d, const real* __restrict__ vs, int obs0, int k, int g) {
  const int n = 9 * k;
  const int c0 = min(4 * g, n - 1), c3 = min(4 * g + 3, n - 1);
  const int oa = (unsigned)c0 / 9u, ob = (unsigned)c3 / 9u;  // at most two observations
  const int ca = 12 * d.obs_cam[obs0 + oa], cb = 12 * d.obs_cam[obs0 + ob];
  real out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = min(4 * g + q, n - 1);
    const int o = (unsigned)c / 9u;
    const int idx = (o == oa ? ca : cb) + (c - 9 * o);
    out[q] = (4 * g + q < n) ? vs[idx] : 0.f;
  }
  return make_real4(out[0], out[1], out[2], out[3]);
}

// A float4 of a landmark block, with a non-temporal load when NT (streamed
// once: no allocation in the caches, which keeps them for the other data of
// the product when the blocks are much larger than the last-level cache).
template <bool NT>
__device__ __forceinline__ real4 load_block(const real4* p) {
  if constexpr (NT) {
    typedef real v4 __attribute__((ext_vector_type(4)));
    const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    return make_real4(v.x, v.y, v.z, v.w);
  } else {
    return *p;
  }
}

__device__ __forceinline__ real dot4(real4 a, real4 b) { return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w; }

__device__ __forceinline__ void axpy4(real4& z, real y, real4 b) {
  z.x += y * b.x;
  z.y += y * b.y;
  z.z += y * b.z;
  z.w += y * b.w;
}

// Store the outputs of column group g: every landmark owns a 16-byte aligned
// region of W floats at obsbuf[slot_zoff] (its 9k outputs, observation-major,
// then padding), written as whole float4s so no cache line is partly written.
__device__ __forceinline__ void store_cols(const Dev& d, int zoff, int g, real4 z) {
  reinterpret_cast<real4*>(d.obsbuf + zoff)[g] = z;
}


// In PCG mode (the template flag PCG) the product skips the landmarks of
// problems whose solve has ended; otherwise every active landmark is done.
//
// Matrix-free product for teams of <= 64 lanes, one landmark per team: one
// float4 column group per lane; for every B row the team forms
// y_r = B_r . p' with a DPP all-reduce and accumulates z += y_r B_r, so each B
// entry is read from memory once.  Rows are taken in batches of RB: the first
// batch is requested before the gather, and each batch before the previous
// one is reduced, so up to 2 RB rows are in flight per lane.  Rows past 2k of
// the last batch re-read row 2k-1 (cached) and are given y = 0.  Writes z
// (unscaled, 9 values per observation) to obsbuf.
template <int TEAM, int RB, bool PCG, bool NT>
__device__ __forceinline__ void matvec_teams(const Dev& d, int s0, int send, const real* __restrict__ v) {
  const int team = threadIdx.x / TEAM;
  const int lane = threadIdx.x % TEAM;
  const int slot = s0 + team;
  if (slot >= send) return;  // uniform over the team
  const int prob = d.slot_prob[slot];
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const int zoff = d.slot_zoff[slot];
  const real4* __restrict__ Bs = reinterpret_cast<const real4*>(d.poolB + d.slot_boff[slot]);
  // While every problem of the PCG solve is still running, the first rows and the
  // camera gather are requested before the problem's flags are tested (all these
  // addresses are in bounds whatever the flags say); once one has stopped, its
  // landmarks are tested first so that their blocks are not read.
  const int act = d.active[prob];
  const int dn = PCG ? d.done[prob] : 0;
  if (PCG && d.pcg_skip[0] && (!act || dn)) return;
  const int G = width_of(k) >> 2, n = 2 * k;
  const real4* __restrict__ Bj = Bs + min(lane, G - 1);
  real4 c[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) c[i] = load_block<NT>(&Bj[(size_t)min(i, n - 1) * G]);
  const real4 pv = lane < G ? gather_cols(d, v, obs0, k, lane) : make_real4(0.f, 0.f, 0.f, 0.f);
  if (!act || dn) return;  // uniform over the team
  real4 z = make_real4(0.f, 0.f, 0.f, 0.f);
  for (int r = 0; r < n; r += RB) {
    const int rn = r + RB;
    real4 nx[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) nx[i] = c[i];
    if (rn < n) {
#pragma unroll
      for (int i = 0; i < RB; ++i) nx[i] = load_block<NT>(&Bj[(size_t)min(rn + i, n - 1) * G]);
    }
    real y[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) y[i] = team_sum<TEAM>(dot4(c[i], pv));
#pragma unroll
    for (int i = 0; i < RB; ++i) axpy4(z, r + i < n ? y[i] : 0.f, c[i]);
#pragma unroll
    for (int i = 0; i < RB; ++i) c[i] = nx[i];
  }
  if (lane < G) store_cols(d, zoff, lane, z);
}

// Matrix-free product for large landmarks: a workgroup of 4 wavefronts per
// landmark.  Wave w takes rows w, w+4, ... in steps of RS rows (w, w+4, ...,
// w+4(RS-1)); each lane owns up to NCG column groups (strided by 64).  The next
// step's rows are requested before the current ones are reduced.  The 4
// partial z vectors are summed through LDS in a fixed order.
template <int NCG, int RS, bool PCG, bool NT>
__device__ __forceinline__ void matvec_large(const Dev& d, int slot, const real* v, real4 (*zred)[64]) {
  const int prob = d.slot_prob[slot];
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const int zoff = d.slot_zoff[slot];
  const real4* __restrict__ B = reinterpret_cast<const real4*>(d.poolB + d.slot_boff[slot]);
  if (!d.active[prob] || (PCG && d.done[prob])) return;
  const int G = width_of(k) >> 2;
  const int n = 2 * k;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  auto load = [&](int r, real4 (&b)[RS][NCG]) {
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int rr = min(r + 4 * i, n - 1);
#pragma unroll
      for (int j = 0; j < NCG; ++j) {
        b[i][j] = make_real4(0.f, 0.f, 0.f, 0.f);
        if (64 * j < G) b[i][j] = load_block<NT>(&B[(size_t)rr * G + min(lane + 64 * j, G - 1)]);
      }
    }
  };
  real4 b[RS][NCG], pv[NCG], z[NCG];
  load(w, b);  // n >= 58 > w
#pragma unroll
  for (int j = 0; j < NCG; ++j) {
    const int g = lane + 64 * j;
    pv[j] = g < G ? gather_cols(d, v, obs0, k, g) : make_real4(0.f, 0.f, 0.f, 0.f);
    z[j] = make_real4(0.f, 0.f, 0.f, 0.f);
  }
  for (int r = w; r < n; r += 4 * RS) {
    real4 nb[RS][NCG];
    if (r + 4 * RS < n) {
      load(r + 4 * RS, nb);
    } else {
#pragma unroll
      for (int i = 0; i < RS; ++i)
#pragma unroll
        for (int j = 0; j < NCG; ++j) nb[i][j] = b[i][j];
    }
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      real y = 0.f;
#pragma unroll
      for (int j = 0; j < NCG; ++j) y += dot4(b[i][j], pv[j]);
      y = wave_sum_f(y);
      if (r + 4 * i >= n) y = 0.f;  // clamped re-read of the last row
#pragma unroll
      for (int j = 0; j < NCG; ++j) axpy4(z[j], y, b[i][j]);
    }
#pragma unroll
    for (int i = 0; i < RS; ++i)
#pragma unroll
      for (int j = 0; j < NCG; ++j) b[i][j] = nb[i][j];
  }
#pragma unroll
  for (int j = 0; j < NCG; ++j) {
    if (64 * j >= G) break;  // uniform across the workgroup
    zred[w][lane] = z[j];
    __syncthreads();
    if (w == 0) {
      const real4 a = zred[0][lane], b2 = zred[1][lane], c = zred[2][lane], e = zred[3][lane];
      const real4 s = make_real4((a.x + b2.x) + (c.x + e.x), (a.y + b2.y) + (c.y + e.y),
                                   (a.z + b2.z) + (c.z + e.z), (a.w + b2.w) + (c.w + e.w));
      const int g = lane + 64 * j;
      if (g < G) store_cols(d, zoff, g, s);
    }
    __syncthreads();
  }
}

// Rows per batch of the small classes (3, 2, 1, 0 in launch order), by the
// tunable row-batch set RBS, and rows per wavefront step of class 4.
__host__ __device__ constexpr int mv_rb(int rbs, int j) { return rbs == 0 ? 4 : (j == 3 ? 6 : 8); }
constexpr int MV_RS = 1;
__host__ __device__ constexpr int mv_per_wg(int j) {  // j: launch-order class index 0..4
  return j == 0 ? 1 : WG / class_team(4 - j);
}

// Workgroup b of the product over the size classes 0..3 (and 4 when LARGE):
// every workgroup belongs to one class, so the product over these landmarks is
// a single kernel with no tail gaps between classes.  Without LARGE the kernel
// holds no class-4 code and needs fewer registers (more resident wavefronts);
// class 4 then runs as its own launch (k_matvec_large).
template <bool PCG, bool LARGE, int RBS, bool NT>
__device__ __forceinline__ void matvec_block(const Dev& d, const ClassGrid& m, int b, const real* v,
                                             real4 (*zred)[64]) {
  if constexpr (LARGE) {
    if (b < m.nblk[0]) { matvec_large<4, MV_RS, PCG, false>(d, m.first[0] + b, v, zred); return; }
    b -= m.nblk[0];
  }
  if (b < m.nblk[1]) { matvec_teams<64, mv_rb(RBS, 0), PCG, NT>(d, m.first[1] + b * mv_per_wg(1), m.end[1], v); return; }
  b -= m.nblk[1];
  if (b < m.nblk[2]) { matvec_teams<32, mv_rb(RBS, 1), PCG, NT>(d, m.first[2] + b * mv_per_wg(2), m.end[2], v); return; }
  b -= m.nblk[2];
  if (b < m.nblk[3]) { matvec_teams<16, mv_rb(RBS, 2), PCG, NT>(d, m.first[3] + b * mv_per_wg(3), m.end[3], v); return; }
  b -= m.nblk[3];
  matvec_teams<8, mv_rb(RBS, 3), PCG, NT>(d, m.first[4] + b * mv_per_wg(4), m.end[4], v);
}

// One launch of the product over classes 0..3 (and 4): one workgroup per
// block, or, PERSIST, a fixed grid whose workgroups take blocks b, b + grid,
// ... in turn (largest landmarks first, so the static round-robin balances).
template <bool PCG, bool LARGE, int RBS, bool PERSIST, bool NT>
__global__ __launch_bounds__(WG) void k_matvec(Dev d, ClassGrid m, int nwork, const real* v) {
  __shared__ real4 zred[LARGE ? 4 : 1][64];
  if constexpr (PERSIST) {
    for (int b = blockIdx.x; b < nwork; b += gridDim.x) matvec_block<PCG, LARGE, RBS, NT>(d, m, b, v, zred);
  } else {
    matvec_block<PCG, LARGE, RBS, NT>(d, m, blockIdx.x, v, zred);
  }
}

// Class 4 on its own: one landmark per workgroup.
template <bool PCG, bool NT>
__global__ __launch_bounds__(WG) void k_matvec_large(Dev d, int slot0, const real* v) {
  __shared__ real4 zred[4][64];
  matvec_large<4, MV_RS, PCG, NT>(d, slot0 + blockIdx.x, v, zred);
}

// The largest landmarks (k at least the tuned edge, 29..512), split into blocks
// of `rows` rows so that a few very large landmarks still spread over the
// whole chip: job j (slot, row block) runs on one workgroup of four wavefronts
// (wave w takes rows w, w+4, ... of the block) and writes its partial z for
// the block; a landmark with a single block writes its outputs directly.
template <bool PCG, bool NT>
__global__ __launch_bounds__(WG) void k_matvec_rows(Dev d, int slot0, int rows, const real* v) {
  constexpr int NCG = 18;  // ceil(width_of(512) / 4 / 64)
  __shared__ real4 zred[4][64];
  const int2 job = d.hjob[blockIdx.x];
  const int slot = job.x;
  const int prob = d.slot_prob[slot];
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const real4* __restrict__ B = reinterpret_cast<const real4*>(d.poolB + d.slot_boff[slot]);
  if (!d.active[prob] || (PCG && d.done[prob])) return;
  const int G = width_of(k) >> 2;
  const int n = 2 * k;
  const int r0 = job.y * rows, r1 = min(n, r0 + rows);
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  real4 b[NCG], pv[NCG], z[NCG];
#pragma unroll
  for (int j = 0; j < NCG; ++j) {
    const int g = lane + 64 * j;
    pv[j] = g < G ? gather_cols(d, v, obs0, k, g) : make_real4(0.f, 0.f, 0.f, 0.f);
    z[j] = make_real4(0.f, 0.f, 0.f, 0.f);
  }
  for (int r = r0 + w; r < r1; r += 4) {
    const real4* row = B + (size_t)r * G + lane;
#pragma unroll
    for (int j = 0; j < NCG; ++j) {
      b[j] = make_real4(0.f, 0.f, 0.f, 0.f);
      if (lane + 64 * j < G) b[j] = load_block<NT>(&row[64 * j]);
    }
    real y = 0.f;
#pragma unroll
    for (int j = 0; j < NCG; ++j) y += dot4(b[j], pv[j]);
    y = wave_sum_f(y);
#pragma unroll
    for (int j = 0; j < NCG; ++j) axpy4(z[j], y, b[j]);
  }
  const bool single = n <= rows;
  real4* dst = single ? reinterpret_cast<real4*>(d.obsbuf + d.slot_zoff[slot])
                       : reinterpret_cast<real4*>(d.zpart + d.hz_off[slot - slot0] + (size_t)job.y * (4 * G));
#pragma unroll
  for (int j = 0; j < NCG; ++j) {
    if (64 * j >= G) break;  // uniform across the workgroup
    zred[w][lane] = z[j];
    __syncthreads();
    if (w == 0) {
      const real4 a = zred[0][lane], b2 = zred[1][lane], c = zred[2][lane], e = zred[3][lane];
      const real4 s = make_real4((a.x + b2.x) + (c.x + e.x), (a.y + b2.y) + (c.y + e.y),
                                   (a.z + b2.z) + (c.z + e.z), (a.w + b2.w) + (c.w + e.w));
      const int g = lane + 64 * j;
      if (g < G) dst[g] = s;
    }
    __syncthreads();
  }
}

// Sum of the row-block partials of every landmark of the row-block kernel with
// more than one block, in block order, into its outputs (one workgroup per
// landmark).
template <bool PCG>
__global__ __launch_bounds__(WG) void k_matvec_combine(Dev d, int slot0, int rows) {
  const int slot = slot0 + blockIdx.x;
  const int prob = d.slot_prob[slot];
  const int k = d.slot_k[slot];
  if (!d.active[prob] || (PCG && d.done[prob])) return;
  const int n = 2 * k;
  if (n <= rows) return;
  const int nblk = (n + rows - 1) / rows;
  const int G = width_of(k) >> 2;
  const real4* __restrict__ src = reinterpret_cast<const real4*>(d.zpart + d.hz_off[blockIdx.x]);
  real4* dst = reinterpret_cast<real4*>(d.obsbuf + d.slot_zoff[slot]);
  for (int g = threadIdx.x; g < G; g += WG) {
    real4 s = src[g];
    for (int r = 1; r < nblk; ++r) {
      const real4 t = src[(size_t)r * G + g];
      s.x += t.x; s.y += t.y; s.z += t.z; s.w += t.w;
    }
    dst[g] = s;
  }
}

// ----------------------------------------------------- PCG vector kernels

// One PCG iteration is three kernels, ordered by the kernel boundaries (no
// grid-wide atomics or fences):
//   product   w = B^T B S z over the landmark blocks (per-observation outputs),
//   k_pcg_q   the sums r.z, r.r of the last update -> convergence test and
//             beta; p = z + beta p, q = A z + beta q (= A p), partial p.q,
//   k_pcg_update  alpha = r.z / p.q; x += alpha p, r -= alpha q, z = M^-1 r,
//             partials r.z, r.r.
// The test needs the sums of every camera of a problem, so in this form it
// runs after the next product, which is wasted once the test succeeds.  With
// Dev::test_sep a fourth kernel, k_pcg_test, takes the test right after each
// update (one wavefront per problem, the same sums and decisions, so the same
// bits); the product after convergence is then skipped, at the price of one
// small launch per iteration.
// Every workgroup that needs a per-problem scalar forms it itself from the
// per-camera FP64 partials with the same fixed-order wavefront tree, so all of
// them hold the same bits.  Per-problem state is written by one designated
// workgroup (the one holding the problem's first camera) and never read back
// in the kernel that writes it; the one exception, the done flag, only ever
// goes from 0 to 1 and every workgroup that reads it makes the same decision
// from the sums it formed itself.  (Waves of one workgroup may read the flag
// before and after it is set; they then take the same exit, since a wave
// that went on finds the test failed and the others' partial sums unused.)

__device__ __forceinline__ double problem_sum(const Dev& d, const double* __restrict__ part, int p, int lane) {
  double s = 0.0;
  const int e = d.prob_cam_off[p + 1];
#pragma unroll 4
  for (int c = d.prob_cam_off[p] + lane; c < e; c += 64) s += part[c];
  return wave_sum_d(s);
}

// Two per-problem sums in one pass (same per-lane order as problem_sum, so each
// is bitwise equal to problem_sum of its array).
__device__ __forceinline__ void problem_sum2(const Dev& d, const double* __restrict__ a, const double* __restrict__ b,
                                             int p, int lane, double& sa, double& sb) {
  sa = sb = 0.0;
  const int e = d.prob_cam_off[p + 1];
#pragma unroll 4
  for (int c = d.prob_cam_off[p] + lane; c < e; c += 64) {
    sa += a[c];
    sb += b[c];
  }
  sa = wave_sum_d(sa);
  sb = wave_sum_d(sb);
}

__device__ __forceinline__ void minv_apply(const real* __restrict__ mi, const real r[9], real z[9]) {
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    real v = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q) v += mi[9 * a + q] * r[q];
    z[a] = v;
  }
}

// x = 0, r = -b, z = M^-1 r (and S z), p = q = 0; per-camera partials r.z (cam_part2), r.r (cam_part3).
// Thread 0 also clears the solve's "some problem stopped" flag (launched with at least one workgroup).
__global__ __launch_bounds__(WG) void k_pcg_init(Dev d) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) d.pcg_skip[0] = 0;
  if (c >= d.NC) return;
  const int prob = d.cam_prob[c];
  double rz = 0.0, rr = 0.0;
  if (d.active[prob]) {
    real r[9], z[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      r[a] = -d.vb[9 * c + a];
      d.vx[9 * c + a] = 0.f;
      d.vr[9 * c + a] = r[a];
      d.vp[9 * c + a] = 0.f;
      d.vq[9 * c + a] = 0.f;
    }
    minv_apply(d.minv + 81 * (size_t)c, r, z);
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      d.vz[9 * c + a] = z[a];
      d.vzs[12 * c + a] = d.s_cam[9 * c + a] * z[a];
      rz += (double)(r[a] * z[a]);
      rr += (double)(r[a] * r[a]);
    }
  }
  d.cam_part2[c] = rz;
  d.cam_part3[c] = rr;
}

// One wavefront per problem: per-problem start scalars.  rz holds r0.z0, so
// the first beta is exactly 1 and p = z0 (p and q start at 0).
__global__ __launch_bounds__(WG) void k_pcg_init_scalars(Dev d) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * (WG / 64) + w;
  if (p < d.P) {  // uniform over the wavefront
    double rz, rr;
    problem_sum2(d, d.cam_part2, d.cam_part3, p, lane, rz, rr);
    if (lane == 0) {
      d.rz[p] = rz;
      d.rr0[p] = rr;
      d.rr[p] = rr;
      d.beta[p] = 0.0;
      d.iters[p] = 0;
      d.qmod[p] = 0.0;  // Q(x_0) = 0
      d.dqmod[p] = 0.0;
      if (!d.active[p]) { d.done[p] = 1; d.pstatus[p] = 4; d.pcg_skip[0] = 1; }
      else if (!(rr > 0.0) || !(rz > 0.0) || !isfinite(rz) || !isfinite(rr)) {
        d.done[p] = 1;
        d.pstatus[p] = (rr == 0.0) ? 3 : 2;
        d.pcg_skip[0] = 1;
      } else { d.done[p] = 0; d.pstatus[p] = 1; }
    }
  }
}

// Convergence test of the last update from its sums: 0 continue, 1 converged,
// 2 breakdown (non-finite or non-positive r.z).
__device__ __forceinline__ int pcg_test(const Dev& d, int p, double rz, double rr) {
  if (!isfinite(rr) || !isfinite(rz)) return 2;
  const double tol = (double)d.pcg_tol;
  if (rr <= tol * tol * d.rr0[p]) return 1;
  if (d.pcg_eta > 0.f) {  // Nash-Sofer: i (Q_i - Q_{i-1}) / Q_i < eta after update i >= 1
    const int i = d.iters[p];
    const double q = d.qmod[p];
    if (i >= 1 && q < 0.0 && (double)i * d.dqmod[p] / q < (double)d.pcg_eta) return 1;
  }
  return rz > 0.0 ? 0 : 2;
}

// Per camera (one workgroup).  The gather takes the camera's observations in
// rounds of 4 per thread: the 4 output positions of a round are requested
// together (and those of the next round before the current values are
// summed), so a camera costs one position latency plus one value latency per
// round.  Wave 0 forms the problem sums while its first positions load.
constexpr int Q_UNROLL = 4;

__device__ __forceinline__ void q_positions(const Dev& d, int i0, int e, int zp[Q_UNROLL]) {
#pragma unroll
  for (int j = 0; j < Q_UNROLL; ++j) {
    const int i = i0 + (int)threadIdx.x + j * WG;
    zp[j] = i < e ? d.cam_zpos[i] : -1;
  }
}

__global__ __launch_bounds__(WG) void k_pcg_q(Dev d) {
  __shared__ real part[4][9];
  __shared__ real pqs[9];
  __shared__ real beta_s;
  __shared__ int go_s;
  const int c = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // the first output positions are requested together with the problem's
  // state (one load latency), the outputs only for a problem still solving
  const int b = d.cam_obs_off[c], e = d.cam_obs_off[c + 1];
  const int prob = d.cam_prob[c];
  int zp[Q_UNROLL];
  q_positions(d, b, e, zp);
  real zc = 0.f, pc = 0.f, qc = 0.f, sc = 0.f;
  if (threadIdx.x < 9) {
    const int idx = 9 * c + threadIdx.x;
    zc = d.vz[idx];
    pc = d.vp[idx];
    qc = d.vq[idx];
    sc = d.s_cam[idx];
  }
  if (!d.active[prob] || d.done[prob]) return;  // see the note at the top of this section
  if (d.test_sep) {  // k_pcg_test has taken the test and formed beta
    if (threadIdx.x == 0) {
      beta_s = (real)d.beta[prob];
      go_s = 1;
    }
  } else if (w == 0) {
    int t = 3;  // 3: the problem's solve has ended (or it is inactive)
    double beta = 0.0;
    {
      double rz, rr;
      problem_sum2(d, d.cam_part2, d.cam_part3, prob, lane, rz, rr);
      t = pcg_test(d, prob, rz, rr);
      beta = rz / d.rz[prob];
      if (lane == 0 && c == d.prob_cam_off[prob]) {  // designated writer of the problem's scalars
        d.rr[prob] = rr;
        if (t) {
          d.done[prob] = 1;
          d.pstatus[prob] = t == 1 ? 0 : 2;
          d.pcg_skip[0] = 1;
        } else {
          d.rz_next[prob] = rz;
          d.beta[prob] = beta;
        }
      }
    }
    if (lane == 0) {
      beta_s = (real)beta;
      go_s = t == 0;
    }
  }
  real acc[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) acc[a] = 0.f;
  if (d.sc) {  // the Schur-complement product is already per camera
    if (threadIdx.x == 0) {
#pragma unroll
      for (int a = 0; a < 9; ++a) acc[a] = d.vy[9 * c + a];
    }
  } else
  for (int i0 = b; i0 < e; i0 += Q_UNROLL * WG) {
    int nz[Q_UNROLL];
    const bool more = i0 + Q_UNROLL * WG < e;  // uniform
    if (more) q_positions(d, i0 + Q_UNROLL * WG, e, nz);
#pragma unroll
    for (int j = 0; j < Q_UNROLL; ++j) {
      if (zp[j] >= 0) {
        if (d.implicit) {  // 4-element aligned rows of 12 elements
          const real4* s4 = reinterpret_cast<const real4*>(d.obsbuf + zp[j]);
          const real4 a0 = s4[0], a1 = s4[1], a2 = s4[2];
          acc[0] += a0.x; acc[1] += a0.y; acc[2] += a0.z; acc[3] += a0.w;
          acc[4] += a1.x; acc[5] += a1.y; acc[6] += a1.z; acc[7] += a1.w;
          acc[8] += a2.x;
        } else {
          const real* src = d.obsbuf + zp[j];
#pragma unroll
          for (int a = 0; a < 9; ++a) acc[a] += src[a];
        }
      }
    }
    if (more) {
#pragma unroll
      for (int j = 0; j < Q_UNROLL; ++j) zp[j] = nz[j];
    }
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) acc[a] = wave_sum_f(acc[a]);
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 9; ++a) part[w][a] = acc[a];
  }
  __syncthreads();
  if (!go_s) return;  // uniform: the solve of this problem has ended
  if (threadIdx.x < 9) {
    const int a = threadIdx.x;
    const int idx = 9 * c + a;
    const real s = (part[0][a] + part[1][a]) + (part[2][a] + part[3][a]);
    const real beta = beta_s;
    const real az = sc * s + (real)d.lambda[prob] * zc;  // (A z) of this camera
    const real pn = zc + beta * pc;
    const real qn = az + beta * qc;
    d.vp[idx] = pn;
    d.vq[idx] = qn;
    pqs[a] = pn * qn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double pq = 0.0;
#pragma unroll
    for (int a = 0; a < 9; ++a) pq += (double)pqs[a];
    d.cam_part[c] = pq;
  }
}

// One thread per (camera, row), UPD_CAMS cameras per workgroup (seven: more
// workgroups shorten this latency-bound kernel; 28 per workgroup took 7% longer).  Wave 0 forms
// alpha = rz / p^T q for each problem that owns cameras of the workgroup
// (alpha = 0 and a breakdown status when p^T q is not positive and finite).
constexpr int UPD_CAMS = 7;
// whole wavefronts: wave 0 forms the problem sums with all 64 lanes
constexpr int UPD_THREADS = (9 * UPD_CAMS + 63) / 64 * 64;
static_assert(UPD_THREADS >= 64 && UPD_THREADS <= WG, "k_pcg_update needs a complete wave 0");

__global__ __launch_bounds__(WG) void k_pcg_update(Dev d) {
  __shared__ real rs[UPD_CAMS][9];
  __shared__ real prz[UPD_CAMS][9];
  __shared__ real prr[UPD_CAMS][9];
  __shared__ real alpha_s[UPD_CAMS];
  const int lc = threadIdx.x / 9, a = threadIdx.x - 9 * (threadIdx.x / 9);
  const int c0 = blockIdx.x * UPD_CAMS;
  const int c = c0 + lc;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool valid = c < d.NC && lc < UPD_CAMS;
  // the done flags of the convergence test just made (by k_pcg_q) go to the
  // host's copy; a breakdown found below is seen by the host one chunk later,
  // when the kernels of that problem have already stopped (with test_sep,
  // k_pcg_test writes the copy after this kernel)
  if (blockIdx.x == 0 && d.done_host && !d.test_sep)
    for (int p = threadIdx.x; p < d.P; p += blockDim.x) d.done_host[p] = d.done[p];
  // loads that do not depend on alpha first
  int prob = 0;
  real xv = 0.f, pv = 0.f, rv = 0.f, qv = 0.f, sv = 0.f, mrow[9];
  const int idx = 9 * c + a;
  if (valid) {
    prob = d.cam_prob[c];
    sv = d.s_cam[idx];
    xv = d.vx[idx];
    pv = d.vp[idx];
    rv = d.vr[idx];
    qv = d.vq[idx];
    const real* mi = d.minv + 81 * (size_t)c + 9 * a;
#pragma unroll
    for (int j = 0; j < 9; ++j) mrow[j] = mi[j];
  }
  if (w == 0) {
    // the problems of cameras c0 .. c0 + UPD_CAMS - 1 form runs; one alpha per run
    const int cl = c0 + lane;
    const bool own = lane < UPD_CAMS && cl < d.NC;
    const int pl = own ? d.cam_prob[cl] : -1;
    const int prev = __shfl_up(pl, 1);
    const bool head = own && (lane == 0 || prev != pl);
    uint64_t heads = __ballot(head);
    while (heads) {
      const int h = __builtin_ctzll(heads);
      heads &= heads - 1;
      const int p = __shfl(pl, h);
      real al = 0.f;
      if (d.active[p] && !d.done[p]) {
        const double pq = problem_sum(d, d.cam_part, p, lane);
        const bool ok = pq > 0.0 && isfinite(pq);
        al = ok ? (real)(d.rz_next[p] / pq) : 0.f;
        const int f = d.prob_cam_off[p];
        if (lane == 0 && f >= c0 && f < c0 + UPD_CAMS) {  // designated writer
          if (ok) {
            d.iters[p] += 1;
            d.rz[p] = d.rz_next[p];
            const double dq = -0.5 * (d.rz_next[p] / pq) * d.rz_next[p];  // -alpha r.z / 2
            d.qmod[p] += dq;
            d.dqmod[p] = dq;
          } else {
            d.done[p] = 1;
            d.pstatus[p] = 2;  // breakdown: x kept
            d.pcg_skip[0] = 1;
          }
        }
        if (!ok) al = 0.f;
      }
      if (own && pl == p) alpha_s[lane] = al;
    }
  }
  __syncthreads();
  bool live = false;
  real r = 0.f, z = 0.f;
  if (valid) {
    const real alpha = alpha_s[lc];
    live = d.active[prob] && alpha != 0.f;
    if (live) {
      d.vx[idx] = xv + alpha * pv;
      r = rv - alpha * qv;
      d.vr[idx] = r;
    }
  }
  if (lc < UPD_CAMS) rs[lc][a] = r;
  __syncthreads();
  if (live) {
#pragma unroll
    for (int j = 0; j < 9; ++j) z += mrow[j] * rs[lc][j];
    d.vz[idx] = z;
    d.vzs[12 * c + a] = sv * z;
  }
  if (lc < UPD_CAMS) {
    prz[lc][a] = r * z;
    prr[lc][a] = r * r;
  }
  __syncthreads();
  if (live && a == 0) {
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      rz += (double)prz[lc][j];
      rr += (double)prr[lc][j];
    }
    d.cam_part2[c] = rz;
    d.cam_part3[c] = rr;
  }
}

// One wavefront per problem, after each update (and after k_pcg_init_scalars)
// when Dev::test_sep: the convergence test of k_pcg_q's wave 0 on the same
// sums, in the same order, with the same writes, and the problem's flag into
// the host's copy.  Taking it twice on the same sums changes nothing.
__global__ __launch_bounds__(WG) void k_pcg_test(Dev d) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * (WG / 64) + w;
  if (p >= d.P) return;  // uniform over the wavefront
  int dn = d.done[p];
  if (d.active[p] && !dn) {
    double rz, rr;
    problem_sum2(d, d.cam_part2, d.cam_part3, p, lane, rz, rr);
    if (lane == 0) {
      const int t = pcg_test(d, p, rz, rr);
      d.rr[p] = rr;
      if (t) {
        d.done[p] = 1;
        d.pstatus[p] = t == 1 ? 0 : 2;
        d.pcg_skip[0] = 1;
        dn = 1;
      } else {
        d.rz_next[p] = rz;
        d.beta[p] = rz / d.rz[p];
      }
    }
  }
  if (lane == 0 && d.done_host) d.done_host[p] = d.active[p] ? dn : 1;
}

// One workgroup, once after the last iteration of a solve: the convergence
// test of the last update of every problem still running (its status stays
// "iteration limit" unless that update reached the tolerance) and its r.r.
__global__ __launch_bounds__(WG) void k_pcg_final(Dev d) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int p = w; p < d.P; p += WG / 64) {
    if (!d.active[p] || d.done[p]) continue;  // uniform over the wavefront
    double rz, rr;
    problem_sum2(d, d.cam_part2, d.cam_part3, p, lane, rz, rr);
    if (lane == 0) {
      const int t = pcg_test(d, p, rz, rr);
      d.rr[p] = rr;
      if (t) {
        d.done[p] = 1;
        d.pstatus[p] = t == 1 ? 0 : 2;
        d.pcg_skip[0] = 1;
      }
    }
  }
}

// ----------------------------------------------------- back-substitution

// Per landmark: damped top rows from the stored undamped rows and the Givens
// rotations, u_top = T^ S dx_p, dx~_l = -R^-1 (Q^1^T r + u_top) (eq. backsub_nm),
// dx_l = S_l dx~_l, and the landmark's share of the predicted decrease of the
// undamped linear model, summed over all its rotated rows:
//   pred_l = -sum u (2 rho + u) + lambda |dx~_l|^2,   u = rows . (S dx_p, dx~_l).
template <int TEAM>
__device__ __forceinline__ void backsub_one(const Dev& d, int slot, int lane, real* red4) {
  static_assert(TEAM <= 64 && TEAM >= 2 * 3, "one wavefront at most; the smallest team holds the rows of k = 3");
  // the landmark's metadata is requested at once; the problem's flag only when
  // some problem is inactive
  const int prob = d.slot_prob[slot];
  const int lm = d.slot_lm[slot];
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const int64_t toff = d.slot_toff[slot], boff = d.slot_boff[slot];
  if (!d.all_active && !d.active[prob]) return;
  const int W = width_of(k);
  const int G = W >> 2;
  const int n = 2 * k;
  const real4* T = reinterpret_cast<const real4*>(d.poolT + toff);
  const real4* B = reinterpret_cast<const real4*>(d.poolB + boff);
  // the first batch of B rows and the rows' residuals are requested before the
  // top-row work: a team has at least 2k lanes, so lane j holds rho of row j
  // and lane 0 later takes them by a team shuffle (rows in batches of BS_RB,
  // the next batch requested before the current one is reduced; rows past 2k
  // re-read row 2k-1 and are not counted)
  constexpr int BS_RB = 8;
  const real* rho = d.rhoB + 2 * (size_t)obs0;
  const real4* __restrict__ Bj = B + min(lane, G - 1);
  real4 c[BS_RB];
#pragma unroll
  for (int i = 0; i < BS_RB; ++i) c[i] = Bj[(size_t)min(i, n - 1) * G];
  const real rho_l = rho[min(lane, n - 1)];
  const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real lam = (real)d.lambda[prob];
  Givens6 Gv;
  real Rh[3][3], qrh[3], dr[3];
  damping_rotations(lmd, sqrt(lam), Gv, Rh, qrh, dr);
  real4 pv = make_real4(0.f, 0.f, 0.f, 0.f);
  real u0 = 0.f, u1 = 0.f, u2 = 0.f;
  if (lane < G) {
    pv = gather_cols(d, d.vzs, obs0, k, lane);
    const real4 t0 = T[lane], t1 = T[G + lane], t2 = T[2 * G + lane];
    real a[3], b[3];
    a[0] = t0.x; a[1] = t1.x; a[2] = t2.x; rotate_column(Gv, a, b);
    u0 += a[0] * pv.x; u1 += a[1] * pv.x; u2 += a[2] * pv.x;
    a[0] = t0.y; a[1] = t1.y; a[2] = t2.y; rotate_column(Gv, a, b);
    u0 += a[0] * pv.y; u1 += a[1] * pv.y; u2 += a[2] * pv.y;
    a[0] = t0.z; a[1] = t1.z; a[2] = t2.z; rotate_column(Gv, a, b);
    u0 += a[0] * pv.z; u1 += a[1] * pv.z; u2 += a[2] * pv.z;
    a[0] = t0.w; a[1] = t1.w; a[2] = t2.w; rotate_column(Gv, a, b);
    u0 += a[0] * pv.w; u1 += a[1] * pv.w; u2 += a[2] * pv.w;
  }
  u0 = tsum<TEAM>(u0, red4);
  u1 = tsum<TEAM>(u1, red4);
  u2 = tsum<TEAM>(u2, red4);
  // R^ dx~ = -(qrh + u), upper triangular
  const real c0 = -(qrh[0] + u0), c1 = -(qrh[1] + u1), c2 = -(qrh[2] + u2);
  const real x2 = c2 / Rh[2][2];
  const real x1 = (c1 - Rh[1][2] * x2) / Rh[1][1];
  const real x0 = (c0 - Rh[0][1] * x1 - Rh[0][2] * x2) / Rh[0][0];
  // predicted decrease: top rows, then the 2k B rows
  double pred = 0.0;
  if (lane == 0) {
    const real ut0 = u0 + Rh[0][0] * x0 + Rh[0][1] * x1 + Rh[0][2] * x2;
    const real ut1 = u1 + Rh[1][1] * x1 + Rh[1][2] * x2;
    const real ut2 = u2 + Rh[2][2] * x2;
    pred = -(double)(ut0 * (2.f * qrh[0] + ut0)) - (double)(ut1 * (2.f * qrh[1] + ut1)) -
           (double)(ut2 * (2.f * qrh[2] + ut2)) + (double)lam * ((double)x0 * x0 + (double)x1 * x1 + (double)x2 * x2);
  }
  for (int r = 0; r < n; r += BS_RB) {
    real4 nx[BS_RB];
#pragma unroll
    for (int i = 0; i < BS_RB; ++i) nx[i] = c[i];
    if (r + BS_RB < n) {
#pragma unroll
      for (int i = 0; i < BS_RB; ++i) nx[i] = Bj[(size_t)min(r + BS_RB + i, n - 1) * G];
    }
    real y[BS_RB], rr[BS_RB];
#pragma unroll
    for (int i = 0; i < BS_RB; ++i) y[i] = tsum<TEAM>(dot4(c[i], pv), red4);
#pragma unroll
    for (int i = 0; i < BS_RB; ++i) rr[i] = team_lane<TEAM>(rho_l, min(r + i, n - 1));
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < BS_RB; ++i)
        if (r + i < n) pred -= (double)(y[i] * (2.f * rr[i] + y[i]));
    }
#pragma unroll
    for (int i = 0; i < BS_RB; ++i) c[i] = nx[i];
  }
  if (lane == 0) {
    const real* sl = lmd + LMD_SL;
    d.dxl[3 * (size_t)lm + 0] = sl[0] * x0;
    d.dxl[3 * (size_t)lm + 1] = sl[1] * x1;
    d.dxl[3 * (size_t)lm + 2] = sl[2] * x2;
    d.lm_part[lm] = pred;
  }
}

// The B-row part of the predicted decrease over rows [rbeg, rend) for one
// wavefront of a four-wavefront workgroup: wave w takes rows rbeg + w,
// rbeg + w + 4, ... in steps of RS rows, the next step's rows requested before
// the current ones are reduced (rows past rend re-read row rend-1 and are not
// counted; lanes past the width read column group G-1 against p' = 0).  Lane 0
// returns the wave's sum in row order.
template <int NCG, int RS>
__device__ __forceinline__ double backsub_b_rows(const real4* __restrict__ B, int G, const real4 (&pv)[NCG],
                                                 const real* __restrict__ rho, int rbeg, int rend, int w, int lane) {
  double pred = 0.0;
  if (rbeg + w >= rend) return pred;  // uniform over the wavefront
  auto load = [&](int r, real4 (&b)[RS][NCG], real (&rh)[RS]) {
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int rr = min(r + 4 * i, rend - 1);
      rh[i] = rho[rr];
#pragma unroll
      for (int j = 0; j < NCG; ++j) {
        b[i][j] = make_real4(0.f, 0.f, 0.f, 0.f);
        if (64 * j < G) b[i][j] = B[(size_t)rr * G + min(lane + 64 * j, G - 1)];
      }
    }
  };
  real4 b[RS][NCG];
  real rh[RS];
  load(rbeg + w, b, rh);
  for (int r = rbeg + w; r < rend; r += 4 * RS) {
    real4 nb[RS][NCG];
    real nrh[RS];
    if (r + 4 * RS < rend) {
      load(r + 4 * RS, nb, nrh);
    } else {
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        nrh[i] = rh[i];
#pragma unroll
        for (int j = 0; j < NCG; ++j) nb[i][j] = b[i][j];
      }
    }
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      real y = 0.f;
#pragma unroll
      for (int j = 0; j < NCG; ++j) y += dot4(b[i][j], pv[j]);
      y = wave_sum_f(y);
      if (lane == 0 && r + 4 * i < rend) pred -= (double)(y * (2.f * rh[i] + y));
    }
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      rh[i] = nrh[i];
#pragma unroll
      for (int j = 0; j < NCG; ++j) b[i][j] = nb[i][j];
    }
  }
  return pred;
}

// The damped top rows of a landmark on wave 0 of its workgroup: u = T^ p' by
// the damping rotations of the undamped top rows, dx~_l, dx_l = S_l dx~_l
// (written), and the top rows' share of the predicted decrease (lane 0).
template <int NCG>
__device__ __forceinline__ double backsub_top(const Dev& d, int slot, int prob, int lm, int G, const real4 (&pv)[NCG],
                                              int lane) {
  const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real lam = (real)d.lambda[prob];
  Givens6 Gv;
  real Rh[3][3], qrh[3], dr[3];
  damping_rotations(lmd, sqrt(lam), Gv, Rh, qrh, dr);
  const real4* T = reinterpret_cast<const real4*>(d.poolT + d.slot_toff[slot]);
  real u0 = 0.f, u1 = 0.f, u2 = 0.f;
#pragma unroll
  for (int j = 0; j < NCG; ++j) {
    const int g = lane + 64 * j;
    if (g < G) {
      const real4 t0 = T[g], t1 = T[G + g], t2 = T[2 * G + g];
      real a[3], b[3];
      a[0] = t0.x; a[1] = t1.x; a[2] = t2.x; rotate_column(Gv, a, b);
      u0 += a[0] * pv[j].x; u1 += a[1] * pv[j].x; u2 += a[2] * pv[j].x;
      a[0] = t0.y; a[1] = t1.y; a[2] = t2.y; rotate_column(Gv, a, b);
      u0 += a[0] * pv[j].y; u1 += a[1] * pv[j].y; u2 += a[2] * pv[j].y;
      a[0] = t0.z; a[1] = t1.z; a[2] = t2.z; rotate_column(Gv, a, b);
      u0 += a[0] * pv[j].z; u1 += a[1] * pv[j].z; u2 += a[2] * pv[j].z;
      a[0] = t0.w; a[1] = t1.w; a[2] = t2.w; rotate_column(Gv, a, b);
      u0 += a[0] * pv[j].w; u1 += a[1] * pv[j].w; u2 += a[2] * pv[j].w;
    }
  }
  u0 = wave_sum_f(u0);
  u1 = wave_sum_f(u1);
  u2 = wave_sum_f(u2);
  const real c0 = -(qrh[0] + u0), c1 = -(qrh[1] + u1), c2 = -(qrh[2] + u2);
  const real x2 = c2 / Rh[2][2];
  const real x1 = (c1 - Rh[1][2] * x2) / Rh[1][1];
  const real x0 = (c0 - Rh[0][1] * x1 - Rh[0][2] * x2) / Rh[0][0];
  double top = 0.0;
  if (lane == 0) {
    const real ut0 = u0 + Rh[0][0] * x0 + Rh[0][1] * x1 + Rh[0][2] * x2;
    const real ut1 = u1 + Rh[1][1] * x1 + Rh[1][2] * x2;
    const real ut2 = u2 + Rh[2][2] * x2;
    top = -(double)(ut0 * (2.f * qrh[0] + ut0)) - (double)(ut1 * (2.f * qrh[1] + ut1)) -
          (double)(ut2 * (2.f * qrh[2] + ut2)) + (double)lam * ((double)x0 * x0 + (double)x1 * x1 + (double)x2 * x2);
    const real* sl = lmd + LMD_SL;
    d.dxl[3 * (size_t)lm + 0] = sl[0] * x0;
    d.dxl[3 * (size_t)lm + 1] = sl[1] * x1;
    d.dxl[3 * (size_t)lm + 2] = sl[2] * x2;
  }
  return top;
}

// Large landmarks (one workgroup of 4 wavefronts): the B rows are split over
// the wavefronts as in the product (wave w takes rows w, w+4, ...), with no
// workgroup barrier per row; wave 0 also forms the damped top-row terms and
// dx~_l.  The four partial predictions are added in a fixed order.
template <int NCG, int RS>
__device__ __forceinline__ void backsub_large(const Dev& d, int slot, double* predw) {
  const int prob = d.slot_prob[slot];
  const int lm = d.slot_lm[slot];
  const int k = d.slot_k[slot];
  const int obs0 = d.slot_obs0[slot];
  const int64_t boff = d.slot_boff[slot];
  if (!d.all_active && !d.active[prob]) return;  // uniform over the workgroup
  const int G = width_of(k) >> 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const real4* __restrict__ B = reinterpret_cast<const real4*>(d.poolB + boff);
  real4 pv[NCG];
#pragma unroll
  for (int j = 0; j < NCG; ++j) {
    const int g = lane + 64 * j;
    pv[j] = g < G ? gather_cols(d, d.vzs, obs0, k, g) : make_real4(0.f, 0.f, 0.f, 0.f);
  }
  const real* rho = d.rhoB + 2 * (size_t)obs0;
  const double pred = backsub_b_rows<NCG, RS>(B, G, pv, rho, 0, 2 * k, w, lane);
  if (lane == 0) predw[w] = pred;
  if (w == 0) {
    const double top = backsub_top<NCG>(d, slot, prob, lm, G, pv, lane);
    if (lane == 0) predw[4] = top;
  }
  __syncthreads();
  if (threadIdx.x == 0) d.lm_part[lm] = predw[4] + ((predw[0] + predw[1]) + (predw[2] + predw[3]));
}

// ---------------------------------------------- per-landmark stage launches
//
// Classes 0..4 of each per-landmark stage run as one launch (class_dispatch);
// class 5 has its own launch.

template <bool IMPLICIT>
struct MargF {
  const Dev& d;
  const uint8_t* mask;
  real* lds;
  real* red;
  template <int TEAM, int CLS>
  __device__ __forceinline__ void run(int slot, int lane, int team) const {
    marginalize_one<TEAM, class_kmax(CLS), IMPLICIT>(d, slot, lane, lds + team * marg_stride(class_kmax(CLS)), red,
                                                     mask);
  }
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }
// LDS of the merged launch: the largest (teams per workgroup) x (floats per team) of classes 0..4
constexpr int MARG_LDS_SMALL =
    cmax(cmax(cmax(32 * marg_stride(class_kmax(0)), 16 * marg_stride(class_kmax(1))),
              cmax(8 * marg_stride(class_kmax(2)), 4 * marg_stride(class_kmax(3)))),
         marg_stride(class_kmax(4)));

template <bool IMPLICIT>
__global__ __launch_bounds__(WG) void k_marginalize(Dev d, ClassGrid m, const uint8_t* mask) {
  __shared__ __align__(alignof(real4)) real lds[MARG_LDS_SMALL];
  __shared__ real red[MARG_RED];
  class_dispatch(m, MargF<IMPLICIT>{d, mask, lds, red});
}

template <bool IMPLICIT>
__global__ __launch_bounds__(WG) void k_marginalize_huge(Dev d, int slot0, const uint8_t* mask) {
  __shared__ __align__(alignof(real4)) real lds[marg_stride(class_kmax(5))];
  __shared__ real red[MARG_RED];
  marginalize_one<256, class_kmax(5), IMPLICIT>(d, slot0 + blockIdx.x, threadIdx.x, lds, red, mask);
}

// Explicit blocks of class 5 in row chunks (qjob: slot, first row | end row << 16):
// a block of up to 1024 x 4608 floats is written by several workgroups, each
// repeating the landmark's QR (O(k)) and writing its rows.
__global__ __launch_bounds__(WG) void k_marginalize_chunks(Dev d, const uint8_t* mask) {
  __shared__ __align__(alignof(real4)) real lds[marg_stride(class_kmax(5))];
  __shared__ real red[MARG_RED];
  const int2 j = d.qjob[blockIdx.x];
  marginalize_one<256, class_kmax(5), false>(d, j.x, threadIdx.x, lds, red, mask, j.y & 0xffff, j.y >> 16);
}

struct DampF {
  const Dev& d;
  const uint8_t* mask;
  real* lds;
  template <int TEAM, int CLS>
  __device__ __forceinline__ void run(int slot, int lane, int team) const {
    damp_one<TEAM>(d, slot, lane, mask, lds + team * damp_lds(TEAM));
  }
};

__global__ __launch_bounds__(WG) void k_damp(Dev d, ClassGrid m, const uint8_t* mask) {
  __shared__ __align__(16) real lds[DAMP_LDS];
  class_dispatch(m, DampF{d, mask, lds});
}

__global__ __launch_bounds__(WG) void k_damp_huge(Dev d, int slot0, const uint8_t* mask) {
  __shared__ __align__(16) real lds[damp_lds(256)];
  damp_one<256>(d, slot0 + blockIdx.x, threadIdx.x, mask, lds);
}

// Classes 4..0 of m (launch order; one landmark per workgroup for class 4).
struct BacksubF {
  const Dev& d;
  real* red4;
  double* predw;
  template <int TEAM, int CLS>
  __device__ __forceinline__ void run(int slot, int lane, int) const {
    if constexpr (TEAM == 256)
      backsub_large<4, 2>(d, slot, predw);
    else
      backsub_one<TEAM>(d, slot, lane, red4);
  }
};

__global__ __launch_bounds__(WG) void k_backsub(Dev d, ClassGrid m) {
  __shared__ real red4[4];
  __shared__ double predw[5];
  class_dispatch(m, BacksubF{d, red4, predw});
}

__global__ __launch_bounds__(WG) void k_backsub_huge(Dev d, int slot0) {
  __shared__ double predw[5];
  backsub_large<18, 1>(d, slot0 + blockIdx.x, predw);
}

// ----------------------------------------------------- update and commit

__device__ __forceinline__ void so3_exp_f(real w0, real w1, real w2, real R[9]) {
  const real th2 = w0 * w0 + w1 * w1 + w2 * w2;
  const real th = sqrt(th2);
  real a, b;
  if (th < 1e-4f) {  // series, accurate to FP32 rounding below 1e-4
    a = 1.0f - th2 / 6.0f;
    b = 0.5f - th2 / 24.0f;
  } else {
    const real sh = sin(0.5f * th);
    a = sin(th) / th;
    b = 2.0f * sh * sh / th2;
  }
  // R = I + a W + b W^2
  const real W[9] = {0.f, -w2, w1, w2, 0.f, -w0, -w1, w0, 0.f};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      real w2ij = 0.f;
#pragma unroll
      for (int q = 0; q < 3; ++q) w2ij += W[3 * i + q] * W[3 * q + j];
      R[3 * i + j] = (i == j ? 1.0f : 0.0f) + a * W[3 * i + j] + b * w2ij;
    }
}

// Tentative state of active problems: R' = Exp(dw) R, t' = t + dt, intrinsics
// additive, with dx_p = S dx~_p; landmarks X' = X + dx_l.
__global__ __launch_bounds__(WG) void k_update(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.NC) {
    const int c = i;
    const real* src = d.cam + 16 * (size_t)c;
    real* dst = d.cam_new + 16 * (size_t)c;
    if (!d.active[d.cam_prob[c]]) {
#pragma unroll
      for (int a = 0; a < 16; ++a) dst[a] = src[a];
    } else {
      real dx[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) dx[a] = d.s_cam[9 * c + a] * d.vx[9 * c + a];
      real E[9], R[9];
      so3_exp_f(dx[0], dx[1], dx[2], E);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          R[3 * a + b] = E[3 * a + 0] * src[0 + b] + E[3 * a + 1] * src[3 + b] + E[3 * a + 2] * src[6 + b];
#pragma unroll
      for (int a = 0; a < 9; ++a) dst[a] = R[a];
#pragma unroll
      for (int a = 0; a < 6; ++a) dst[9 + a] = src[9 + a] + dx[3 + a];
      dst[15] = 0.f;
    }
  }
  if (i < d.NL) {
    const real4 X = d.pts[i];
    real4 Y = X;
    if (d.active[d.lm_prob[i]] && d.lm_slot[i] >= 0) {
      Y.x += d.dxl[3 * (size_t)i + 0];
      Y.y += d.dxl[3 * (size_t)i + 1];
      Y.z += d.dxl[3 * (size_t)i + 2];
    }
    d.pts_new[i] = Y;
  }
}

// Keep the tentative state of problems with active && flag (accepted).
__global__ __launch_bounds__(WG) void k_commit(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.NC) {
    const int p = d.cam_prob[i];
    if (d.active[p] && d.flag[p]) {
#pragma unroll
      for (int a = 0; a < 16; ++a) d.cam[16 * (size_t)i + a] = d.cam_new[16 * (size_t)i + a];
    }
  }
  if (i < d.NL) {
    const int p = d.lm_prob[i];
    if (d.active[p] && d.flag[p]) d.pts[i] = d.pts_new[i];
  }
}

// ----------------------------------------------------- test helpers

__global__ __launch_bounds__(WG) void k_debug_lin(Dev d, real* r, real* Jp, real* Jl) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= d.NO) return;
  Cam C;
  load_cam(d.cam, d.obs_cam[o], C);
  const real4 X = d.pts[d.obs_lm[o]];
  const real2 uv = d.obs_uv[o];
  real rr[2], J[2][9], L[2][3];
  project<true>(C, X.x, X.y, X.z, uv.x, uv.y, rr, J, L);
  real sw;  // the rows the QR consumes (Huber IRLS weight applied)
  (void)robust_term(rr[0] * rr[0] + rr[1] * rr[1], d.huber, sw);
  rr[0] *= sw;
  rr[1] *= sw;
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 9; ++b) J[a][b] *= sw;
    for (int b = 0; b < 3; ++b) L[a][b] *= sw;
  }
  r[2 * (size_t)o] = rr[0];
  r[2 * (size_t)o + 1] = rr[1];
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 9; ++b) Jp[18 * (size_t)o + 9 * a + b] = J[a][b];
    for (int b = 0; b < 3; ++b) Jl[6 * (size_t)o + 3 * a + b] = L[a][b];
  }
}

// out = S sum_obs z + lambda v_scaled (no PCG state involved)
__global__ __launch_bounds__(64) void k_cam_gather_product(Dev d, const real* v, real* out) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  real acc[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) acc[a] = 0.f;
  if (d.sc) {
    if (lane == 0) {
#pragma unroll
      for (int a = 0; a < 9; ++a) acc[a] = d.vy[9 * c + a];
    }
  } else {
    for (int i = d.cam_obs_off[c] + lane; i < d.cam_obs_off[c + 1]; i += 64) {
      const real* src = d.obsbuf + d.cam_zpos[i];
#pragma unroll
      for (int a = 0; a < 9; ++a) acc[a] += src[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) acc[a] = wave_sum_f(acc[a]);
  if (lane < 9) {
    real s = acc[0];
#pragma unroll
    for (int a = 1; a < 9; ++a) s = (lane == a) ? acc[a] : s;
    const int idx = 9 * c + lane;
    out[idx] = d.s_cam[idx] * s + (real)d.lambda[d.cam_prob[c]] * v[idx];
  }
}

// ----------------------------------------------- implicit landmark blocks
//
// With implicit blocks the rows of B are never formed.  The six damping
// rotations G of Sec. 5.3 map the top rows [I_3; 0] of the landmark's thin
// factor to [T; N]: T the damped top rows, N the three damping rows, and
// T^T T + N^T N = I since G is orthogonal.  The B rows of the explicit form are
// [Q2^T J_p; N Q1^T J_p], so in scaled pose coordinates
//   B^T B   = J_p^T (I - Q1 Q1^T + Q1 D Q1^T) J_p,
//   B^T rho = J_p^T (I - Q1 Q1^T + Q1 D Q1^T) r,      D = N^T N,
// which is the landmark term of eq. red_H / red_b taken from the QR of J_l,
// never from its normal equations.  D = lambda (R1 R1^T + lambda I)^-1 is small
// when lambda is small, so it is kept as its own term: forming I - D first
// would leave the damping part at the level of FP32 rounding of an O(1)
// number.  Each observation carries its record (pose Jacobian rows, its two
// rows of Q1, residual), so every stage below is O(k) per landmark.

// Per landmark (one thread): the damped factors (as the explicit damping) and
// D = N^T N, N the images of the unit columns under the damping rotations.
__global__ __launch_bounds__(WG) void k_damp_implicit(Dev d, const uint8_t* mask) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= d.NS) return;
  const int prob = d.slot_prob[slot];
  if (mask && !mask[prob]) return;
  real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real lam = (real)d.lambda[prob];
  Givens6 Gv;
  real Rh[3][3], qrh[3], dr[3];
  damping_rotations(lmd, sqrt(lam), Gv, Rh, qrh, dr);
  lmd[LMD_RH + 0] = Rh[0][0]; lmd[LMD_RH + 1] = Rh[0][1]; lmd[LMD_RH + 2] = Rh[0][2];
  lmd[LMD_RH + 3] = Rh[1][1]; lmd[LMD_RH + 4] = Rh[1][2]; lmd[LMD_RH + 5] = Rh[2][2];
  lmd[LMD_QRH + 0] = qrh[0]; lmd[LMD_QRH + 1] = qrh[1]; lmd[LMD_QRH + 2] = qrh[2];
  lmd[LMD_LAM] = lam;
  // column j of N: the damping rows of the rotated unit column e_j
  real N[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    real t[3] = {j == 0 ? 1.f : 0.f, j == 1 ? 1.f : 0.f, j == 2 ? 1.f : 0.f}, dd[3];
    rotate_column(Gv, t, dd);
    N[0][j] = dd[0]; N[1][j] = dd[1]; N[2][j] = dd[2];
  }
  real D[6];
  int e = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) D[e++] = N[0][a] * N[0][b] + N[1][a] * N[1][b] + N[2][a] * N[2][b];
  reinterpret_cast<real4*>(lmd + LMD_P)[0] = make_real4(D[0], D[1], D[2], D[3]);
  reinterpret_cast<real2*>(lmd + LMD_P + 4)[0] = make_real2(D[4], D[5]);
}

__device__ __forceinline__ void load_p(const real* lmd, real P[3][3]) {
  const real4 a = reinterpret_cast<const real4*>(lmd + LMD_P)[0];
  const real2 b = reinterpret_cast<const real2*>(lmd + LMD_P + 4)[0];
  P[0][0] = a.x; P[0][1] = P[1][0] = a.y; P[0][2] = P[2][0] = a.z;
  P[1][1] = a.w; P[1][2] = P[2][1] = b.x; P[2][2] = b.y;
}

// The pose Jacobian rows (2 x 9) and Q1 rows (2 x 3) of record i.
__device__ __forceinline__ void load_rec(const Dev& d, int i, real (&J)[2][9], real (&Q)[2][3]) {
  const real4* rec = rec_plane(d, 0) + i;
  const size_t P = (size_t)d.NO;
  const real4 a = rec[0], b = rec[P], c = rec[2 * P], e = rec[3 * P], f = rec[4 * P], g = rec[5 * P];
  J[0][0] = a.x; J[0][1] = a.y; J[0][2] = a.z; J[0][3] = a.w; J[0][4] = b.x; J[0][5] = b.y; J[0][6] = b.z;
  J[0][7] = b.w; J[0][8] = c.x;
  J[1][0] = c.y; J[1][1] = c.z; J[1][2] = c.w; J[1][3] = e.x; J[1][4] = e.y; J[1][5] = e.z; J[1][6] = e.w;
  J[1][7] = f.x; J[1][8] = f.y;
  Q[0][0] = f.z; Q[0][1] = f.w; Q[0][2] = g.x;
  Q[1][0] = g.y; Q[1][1] = g.z; Q[1][2] = g.w;
}

// Per observation (one thread): its block-Jacobi terms G = J_o^T Pi J_o (45 upper
// entries, Pi = (I - Q1o Q1o^T) + Q1o D Q1o^T the observation's 2 x 2 block of the
// projector) and right-hand side g = J_o^T ((r_o - Q1o Q1^T r) + Q1o D Q1^T r),
// unscaled, to obsbuf[obs][0..53] (the layout of the explicit pass).
__global__ __launch_bounds__(WG) void k_precond_obs_implicit(Dev d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d.NO) return;
  const int slot = d.lm_slot[d.obs_lm[q]];
  const int prob = d.slot_prob[slot];
  if (!d.active[prob]) return;
  const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const int ri = d.slot_zoff[slot] + (q - d.slot_obs0[slot]);
  real D[3][3], J[2][9], Q[2][3];
  load_p(lmd, D);
  load_rec(d, ri, J, Q);
  const real4 rv = rec_plane(d, 6)[ri];
  const real qr[3] = {lmd[LMD_QR + 0], lmd[LMD_QR + 1], lmd[LMD_QR + 2]};
  real DQ[2][3], Dqr[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    DQ[0][a] = D[a][0] * Q[0][0] + D[a][1] * Q[0][1] + D[a][2] * Q[0][2];
    DQ[1][a] = D[a][0] * Q[1][0] + D[a][1] * Q[1][1] + D[a][2] * Q[1][2];
    Dqr[a] = D[a][0] * qr[0] + D[a][1] * qr[1] + D[a][2] * qr[2];
  }
  real Pi[2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const real proj = (h == h2 ? 1.f : 0.f) - (Q[h][0] * Q[h2][0] + Q[h][1] * Q[h2][1] + Q[h][2] * Q[h2][2]);
      Pi[h][h2] = proj + (Q[h][0] * DQ[h2][0] + Q[h][1] * DQ[h2][1] + Q[h][2] * DQ[h2][2]);
    }
  real rp[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const real rq = (h == 0 ? rv.x : rv.y) - (Q[h][0] * qr[0] + Q[h][1] * qr[1] + Q[h][2] * qr[2]);
    rp[h] = rq + (Q[h][0] * Dqr[0] + Q[h][1] * Dqr[1] + Q[h][2] * Dqr[2]);
  }
  real K[2][9];  // Pi J
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < 9; ++b) K[h][b] = Pi[h][0] * J[0][b] + Pi[h][1] * J[1][b];
  real* out = d.obsbuf + (size_t)q * 54;
  int e = 0;
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int b = a; b < 9; ++b) out[e++] = J[0][a] * K[0][b] + J[1][a] * K[1][b];
#pragma unroll
  for (int a = 0; a < 9; ++a) out[45 + a] = J[0][a] * rp[0] + J[1][a] * rp[1];
}

// Launch description of all six classes for the implicit kernels, launch order
// 5, 4, 3, 2, 1, 0; teams of 64, 64, 32, 16, 8, 4 lanes with 8, 2, 1, 1, 1, 1
// observations per lane.
struct ImplGrid {
  int nblk[6];
  int first[6];
  int end[6];
};
__host__ __device__ constexpr int impl_team(int j) { return j <= 1 ? 64 : 128 >> j; }

template <class F>
__device__ __forceinline__ void impl_dispatch(const ImplGrid& m, const F& f) {
  int b = blockIdx.x;
#define SQRTBA_IMPL_CASE(J, TEAM, OPL)                                             \
  if (b < m.nblk[J]) {                                                           \
    const int t = threadIdx.x / TEAM, slot = m.first[J] + b * (WG / TEAM) + t;   \
    if (slot < m.end[J]) f.template run<TEAM, OPL>(slot, threadIdx.x % TEAM);    \
    return;                                                                      \
  }                                                                              \
  b -= m.nblk[J];
  SQRTBA_IMPL_CASE(0, 64, 8)
  SQRTBA_IMPL_CASE(1, 64, 2)
  SQRTBA_IMPL_CASE(2, 32, 1)
  SQRTBA_IMPL_CASE(3, 16, 1)
  SQRTBA_IMPL_CASE(4, 8, 1)
  SQRTBA_IMPL_CASE(5, 4, 1)
#undef SQRTBA_IMPL_CASE
}

// Product for one landmark: u_o = J_o p'_o per observation (p' = S z, gathered
// from vzs), c = Q1^T u (team sum), e = D c,
// z_o = J_o^T ((u_o - Q1o c) + Q1o e), written as 12 floats (3 float4, the last 3
// zero) per record.  Teams with at most two observations per lane keep their
// records in registers; the others read them again (from cache) after the sum.
template <int TEAM, int OPL, bool PCG>
__device__ __forceinline__ void matvec_implicit(const Dev& d, int slot, int lane) {
  constexpr bool KEEP = OPL <= 2;
  const int prob = d.slot_prob[slot];
  const int k = d.slot_k[slot];
  const int r0 = d.slot_zoff[slot];
  // the records of the lane's first observations are requested before the
  // problem's flags are tested while every problem of the PCG solve is running
  // (in bounds whatever the flags say), after the test once one has stopped
  const int act = d.active[prob];
  const int dn = PCG ? d.done[prob] : 0;
  if (PCG && d.pcg_skip[0] && (!act || dn)) return;
  real u[OPL][2];
  real J[OPL][2][9], Q[OPL][2][3];
  int cm[OPL];
#pragma unroll
  for (int m = 0; m < (KEEP ? OPL : 1); ++m) {
    const int o = lane + TEAM * m;
    if (o < k) {
      cm[m] = d.rec_cam[r0 + o];
      load_rec(d, r0 + o, J[m], Q[m]);
    }
  }
  if (!act || dn) return;  // uniform over the team
  real c[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    u[m][0] = u[m][1] = 0.f;
    if (o < k) {
      if (m >= (KEEP ? OPL : 1)) {
        cm[m] = d.rec_cam[r0 + o];
        load_rec(d, r0 + o, J[m], Q[m]);
      }
      const real4* vs = reinterpret_cast<const real4*>(d.vzs) + 3 * (size_t)cm[m];
      const real4 v0 = vs[0], v1 = vs[1], v2 = vs[2];
      const real pa[9] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x};
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        u[m][0] += J[m][0][a] * pa[a];
        u[m][1] += J[m][1][a] * pa[a];
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) c[j] += Q[m][0][j] * u[m][0] + Q[m][1][j] * u[m][1];
    }
  }
  int buf = 0;
  team_sum_n<TEAM, 3>(c, nullptr, buf);
  real D[3][3];
  load_p(d.lmd + (size_t)slot * LMD_STRIDE, D);
  const real e[3] = {D[0][0] * c[0] + D[0][1] * c[1] + D[0][2] * c[2], D[1][0] * c[0] + D[1][1] * c[1] + D[1][2] * c[2],
                      D[2][0] * c[0] + D[2][1] * c[1] + D[2][2] * c[2]};
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    if (o < k) {
      if constexpr (!KEEP) load_rec(d, r0 + o, J[m], Q[m]);
      const real t0 = u[m][0] - (Q[m][0][0] * c[0] + Q[m][0][1] * c[1] + Q[m][0][2] * c[2]);
      const real t1 = u[m][1] - (Q[m][1][0] * c[0] + Q[m][1][1] * c[1] + Q[m][1][2] * c[2]);
      const real w0 = t0 + (Q[m][0][0] * e[0] + Q[m][0][1] * e[1] + Q[m][0][2] * e[2]);
      const real w1 = t1 + (Q[m][1][0] * e[0] + Q[m][1][1] * e[1] + Q[m][1][2] * e[2]);
      real z[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) z[a] = J[m][0][a] * w0 + J[m][1][a] * w1;
      real4* out = reinterpret_cast<real4*>(d.obsbuf) + 3 * (size_t)(r0 + o);
      out[0] = make_real4(z[0], z[1], z[2], z[3]);
      out[1] = make_real4(z[4], z[5], z[6], z[7]);
      out[2] = make_real4(z[8], 0.f, 0.f, 0.f);
    }
  }
}

template <bool PCG>
struct MatvecImplF {
  const Dev& d;
  template <int TEAM, int OPL>
  __device__ __forceinline__ void run(int slot, int lane) const { matvec_implicit<TEAM, OPL, PCG>(d, slot, lane); }
};

template <bool PCG>
__global__ __launch_bounds__(WG) void k_matvec_implicit(Dev d, ImplGrid m) {
  impl_dispatch(m, MatvecImplF<PCG>{d});
}

// vzs = S v (12 floats per camera, the pad stays zero): the gathered vector of a
// product outside PCG, and S dx_p for the explicit back-substitution.
__global__ __launch_bounds__(WG) void k_prescale(Dev d, const real* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * d.NC) return;
  const int c = i / 9, a = i - 9 * c;
  d.vzs[12 * c + a] = d.s_cam[i] * v[i];
}

// Back-substitution for one landmark: u = J_p p' (p' = S dx_p), c = Q1^T u, the
// damped top rows T^ p' and damping rows D p' by the Givens rotations of c,
// dx~_l = -Rh^-1 (Q^1^T r + T^ p') (eq. backsub_nm), and the model decrease over
// the rotated rows: top rows as in the explicit form, and for the B rows
// sum u (2 rho + u) = 2 (u'.r + d.dr) + |u'|^2 + |d|^2 with u' = u - Q1 c.
template <int TEAM, int OPL>
__device__ __forceinline__ void backsub_implicit(const Dev& d, int slot, int lane) {
  const int prob = d.slot_prob[slot];
  const int lm = d.slot_lm[slot];
  if (!d.active[prob]) return;  // uniform over the team
  const int k = d.slot_k[slot];
  const int r0 = d.slot_zoff[slot];
  const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real lam = (real)d.lambda[prob];
  real u[OPL][2];
  real c[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    u[m][0] = u[m][1] = 0.f;
    if (o < k) {
      real J[2][9], Q[2][3];
      load_rec(d, r0 + o, J, Q);
      const int cam = 9 * d.rec_cam[r0 + o];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const real pa = d.s_cam[cam + a] * d.vx[cam + a];
        u[m][0] += J[0][a] * pa;
        u[m][1] += J[1][a] * pa;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) c[j] += Q[0][j] * u[m][0] + Q[1][j] * u[m][1];
    }
  }
  int buf = 0;
  team_sum_n<TEAM, 3>(c, nullptr, buf);
  real s2[2] = {0.f, 0.f};  // |u'|^2, u'.r
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    if (o < k) {
      real J[2][9], Q[2][3];
      load_rec(d, r0 + o, J, Q);
      const real4 rv = rec_plane(d, 6)[r0 + o];
      const real w0 = u[m][0] - (Q[0][0] * c[0] + Q[0][1] * c[1] + Q[0][2] * c[2]);
      const real w1 = u[m][1] - (Q[1][0] * c[0] + Q[1][1] * c[1] + Q[1][2] * c[2]);
      s2[0] += w0 * w0 + w1 * w1;
      s2[1] += w0 * rv.x + w1 * rv.y;
    }
  }
  team_sum_n<TEAM, 2>(s2, nullptr, buf);
  if (lane == 0) {
    Givens6 Gv;
    real Rh[3][3], qrh[3], dr[3];
    damping_rotations(lmd, sqrt(lam), Gv, Rh, qrh, dr);
    real t[3] = {c[0], c[1], c[2]}, dd[3];
    rotate_column(Gv, t, dd);  // t = T^ p', dd = D p'
    const real c0 = -(qrh[0] + t[0]), c1 = -(qrh[1] + t[1]), c2 = -(qrh[2] + t[2]);
    const real x2 = c2 / Rh[2][2];
    const real x1 = (c1 - Rh[1][2] * x2) / Rh[1][1];
    const real x0 = (c0 - Rh[0][1] * x1 - Rh[0][2] * x2) / Rh[0][0];
    const real ut0 = t[0] + Rh[0][0] * x0 + Rh[0][1] * x1 + Rh[0][2] * x2;
    const real ut1 = t[1] + Rh[1][1] * x1 + Rh[1][2] * x2;
    const real ut2 = t[2] + Rh[2][2] * x2;
    double pred = -(double)(ut0 * (2.f * qrh[0] + ut0)) - (double)(ut1 * (2.f * qrh[1] + ut1)) -
                  (double)(ut2 * (2.f * qrh[2] + ut2)) + (double)lam * ((double)x0 * x0 + (double)x1 * x1 + (double)x2 * x2);
    const double ddr = (double)dd[0] * dr[0] + (double)dd[1] * dr[1] + (double)dd[2] * dr[2];
    const double dd2 = (double)dd[0] * dd[0] + (double)dd[1] * dd[1] + (double)dd[2] * dd[2];
    pred -= 2.0 * ((double)s2[1] + ddr) + (double)s2[0] + dd2;
    const real* sl = lmd + LMD_SL;
    d.dxl[3 * (size_t)lm + 0] = sl[0] * x0;
    d.dxl[3 * (size_t)lm + 1] = sl[1] * x1;
    d.dxl[3 * (size_t)lm + 2] = sl[2] * x2;
    d.lm_part[lm] = pred;
  }
}

struct BacksubImplF {
  const Dev& d;
  template <int TEAM, int OPL>
  __device__ __forceinline__ void run(int slot, int lane) const { backsub_implicit<TEAM, OPL>(d, slot, lane); }
};

__global__ __launch_bounds__(WG) void k_backsub_implicit(Dev d, ImplGrid m) { impl_dispatch(m, BacksubImplF{d}); }

// ------------------------------------------ explicit Schur complement (FP32)
//
// The comparator of the paper's explicit solver (Sec. 4.2, eq. red_normal_eq):
// per landmark the normal-equation blocks H_ll = (J_l S_l)^T (J_l S_l) and
// b_l = (J_l S_l)^T r, per observation G_o = J_o^T (J_lo S_l), and the reduced
// camera matrix H_pp - sum_l G H~_ll^-1 G^T assembled in FP32 as 9 x 9 blocks
// per camera pair, H~_ll = H_ll + lambda I.  Pose columns stay unscaled as in
// the square-root path (S_p is applied where the vectors are gathered), so the
// preconditioner, the PCG vector kernels and the LM loop are shared.

// Float f (0..27) of record i: planes of 4 floats, plane-major.
__device__ __forceinline__ real rec_float(const Dev& d, int i, int f) {
  return d.obsrec[4 * ((size_t)(f >> 2) * d.NO + i) + (f & 3)];
}

// Per landmark: linearize its observations (with the Huber weight), store the
// records (J_p, unscaled J_l, r), and the scaled H_ll, b_l and landmark scales.
template <int TEAM, int OPL>
__device__ __forceinline__ void sc_prepare(const Dev& d, int slot, int lane, const uint8_t* mask) {
  const int prob = d.slot_prob[slot];
  if (mask && !mask[prob]) return;
  const int k = d.slot_k[slot], obs0 = d.slot_obs0[slot], r0 = d.slot_zoff[slot];
  const real4 X = d.pts[d.slot_lm[slot]];
  real h[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // H_ll upper (6), b_l (3), unscaled
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    if (o < k) {
      Cam C;
      load_cam(d.cam, d.obs_cam[obs0 + o], C);
      const real2 uv = d.obs_uv[obs0 + o];
      real r[2], Jp[2][9], Jl[2][3];
      project<true>(C, X.x, X.y, X.z, uv.x, uv.y, r, Jp, Jl);
      real sw;
      (void)robust_term(r[0] * r[0] + r[1] * r[1], d.huber, sw);
      r[0] *= sw;
      r[1] *= sw;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        Jp[0][j] *= sw;
        Jp[1][j] *= sw;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        Jl[0][j] *= sw;
        Jl[1][j] *= sw;
      }
      int e = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) h[e++] += Jl[0][a] * Jl[0][b] + Jl[1][a] * Jl[1][b];
#pragma unroll
      for (int a = 0; a < 3; ++a) h[6 + a] += Jl[0][a] * r[0] + Jl[1][a] * r[1];
      real4* rec = rec_plane(d, 0) + r0 + o;
      const size_t P = (size_t)d.NO;
      rec[0] = make_real4(Jp[0][0], Jp[0][1], Jp[0][2], Jp[0][3]);
      rec[P] = make_real4(Jp[0][4], Jp[0][5], Jp[0][6], Jp[0][7]);
      rec[2 * P] = make_real4(Jp[0][8], Jp[1][0], Jp[1][1], Jp[1][2]);
      rec[3 * P] = make_real4(Jp[1][3], Jp[1][4], Jp[1][5], Jp[1][6]);
      rec[4 * P] = make_real4(Jp[1][7], Jp[1][8], Jl[0][0], Jl[0][1]);
      rec[5 * P] = make_real4(Jl[0][2], Jl[1][0], Jl[1][1], Jl[1][2]);
      rec[6 * P] = make_real4(r[0], r[1], 0.f, 0.f);
    }
  }
  int buf = 0;
  team_sum_n<TEAM, 9>(h, nullptr, buf);
  if (lane == 0) {
    // unit-norm landmark columns (an empty column keeps scale 1), then S_l H S_l, S_l b
    const real s0 = h[0] > 0.f ? 1.0f / sqrt(h[0]) : 1.0f;
    const real s1 = h[3] > 0.f ? 1.0f / sqrt(h[3]) : 1.0f;
    const real s2 = h[5] > 0.f ? 1.0f / sqrt(h[5]) : 1.0f;
    real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
    lmd[LMD_R + 0] = s0 * h[0] * s0; lmd[LMD_R + 1] = s0 * h[1] * s1; lmd[LMD_R + 2] = s0 * h[2] * s2;
    lmd[LMD_R + 3] = s1 * h[3] * s1; lmd[LMD_R + 4] = s1 * h[4] * s2; lmd[LMD_R + 5] = s2 * h[5] * s2;
    lmd[LMD_QR + 0] = s0 * h[6]; lmd[LMD_QR + 1] = s1 * h[7]; lmd[LMD_QR + 2] = s2 * h[8];
    lmd[LMD_SL + 0] = s0; lmd[LMD_SL + 1] = s1; lmd[LMD_SL + 2] = s2;
  }
}

template <bool UNUSED>
struct ScPrepF {
  const Dev& d;
  const uint8_t* mask;
  template <int TEAM, int OPL>
  __device__ __forceinline__ void run(int slot, int lane) const { sc_prepare<TEAM, OPL>(d, slot, lane, mask); }
};

__global__ __launch_bounds__(WG) void k_sc_prepare(Dev d, ImplGrid m, const uint8_t* mask) {
  impl_dispatch(m, ScPrepF<true>{d, mask});
}

// Per landmark: (H_ll + lambda I)^-1 by a 3 x 3 Cholesky factorization in FP32
// (a non-positive pivot, possible only at lambda = 0 for a rank-deficient J_l,
// drops the landmark: inverse 0).
__global__ __launch_bounds__(WG) void k_sc_damp(Dev d, const uint8_t* mask) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= d.NS) return;
  const int prob = d.slot_prob[slot];
  if (mask && !mask[prob]) return;
  real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real lam = (real)d.lambda[prob];
  const real a00 = lmd[LMD_R + 0] + lam, a01 = lmd[LMD_R + 1], a02 = lmd[LMD_R + 2];
  const real a11 = lmd[LMD_R + 3] + lam, a12 = lmd[LMD_R + 4], a22 = lmd[LMD_R + 5] + lam;
  real P[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const real l00 = a00 > 0.f ? sqrt(a00) : 0.f;
  if (l00 > 0.f) {
    const real l10 = a01 / l00, l20 = a02 / l00;
    const real d11 = a11 - l10 * l10;
    const real l11 = d11 > 0.f ? sqrt(d11) : 0.f;
    if (l11 > 0.f) {
      const real l21 = (a12 - l20 * l10) / l11;
      const real d22 = a22 - l20 * l20 - l21 * l21;
      const real l22 = d22 > 0.f ? sqrt(d22) : 0.f;
      if (l22 > 0.f) {
        // L^-1 (lower), then A^-1 = L^-T L^-1
        const real i00 = 1.0f / l00, i11 = 1.0f / l11, i22 = 1.0f / l22;
        const real i10 = -l10 * i00 * i11;
        const real i21 = -l21 * i11 * i22;
        const real i20 = -(l20 * i00 + l21 * i10) * i22;
        P[0] = i00 * i00 + i10 * i10 + i20 * i20;
        P[1] = i10 * i11 + i20 * i21;
        P[2] = i20 * i22;
        P[3] = i11 * i11 + i21 * i21;
        P[4] = i21 * i22;
        P[5] = i22 * i22;
      }
    }
  }
  reinterpret_cast<real4*>(lmd + LMD_P)[0] = make_real4(P[0], P[1], P[2], P[3]);
  reinterpret_cast<real2*>(lmd + LMD_P + 4)[0] = make_real2(P[4], P[5]);
  lmd[LMD_LAM] = lam;
}

// G = J_p^T (J_l S_l) (9 x 3) of record i, and the record's pose Jacobian rows.
__device__ __forceinline__ void sc_load_g(const Dev& d, int i, const real sl[3], real (&J)[2][9], real (&G)[9][3]) {
  real Lu[2][3];
  load_rec(d, i, J, Lu);
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int m = 0; m < 3; ++m) G[a][m] = (J[0][a] * Lu[0][m] + J[1][a] * Lu[1][m]) * sl[m];
}

// Per observation (one thread, landmark order): its block-Jacobi terms
// J^T J - G H~^-1 G^T (45 upper entries) and right-hand side J^T r - G H~^-1 b_l
// to obsbuf[obs][0..53], the layout the per-camera preconditioner sums.
__global__ __launch_bounds__(WG) void k_sc_precond_obs(Dev d) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= d.NO) return;
  const int slot = d.lm_slot[d.obs_lm[q]];
  if (!d.active[d.slot_prob[slot]]) return;
  const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const int ri = d.slot_zoff[slot] + (q - d.slot_obs0[slot]);
  const real sl[3] = {lmd[LMD_SL + 0], lmd[LMD_SL + 1], lmd[LMD_SL + 2]};
  real Hi[3][3], J[2][9], G[9][3];
  load_p(lmd, Hi);
  sc_load_g(d, ri, sl, J, G);
  const real4 rv = rec_plane(d, 6)[ri];
  const real bl[3] = {lmd[LMD_QR + 0], lmd[LMD_QR + 1], lmd[LMD_QR + 2]};
  real T[9][3];  // G H~^-1
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int n = 0; n < 3; ++n) T[a][n] = G[a][0] * Hi[0][n] + G[a][1] * Hi[1][n] + G[a][2] * Hi[2][n];
  real* out = d.obsbuf + (size_t)q * 54;
  int e = 0;
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int b = a; b < 9; ++b)
      out[e++] = J[0][a] * J[0][b] + J[1][a] * J[1][b] - (T[a][0] * G[b][0] + T[a][1] * G[b][1] + T[a][2] * G[b][2]);
#pragma unroll
  for (int a = 0; a < 9; ++a)
    out[45 + a] = J[0][a] * rv.x + J[1][a] * rv.y - (T[a][0] * bl[0] + T[a][1] * bl[1] + T[a][2] * bl[2]);
}

// Off-diagonal block b, row i (one thread): -sum over the block's contributions
// (records a, b of one landmark) of (G_a H~^-1 G_b^T) row i, in list order.
__global__ __launch_bounds__(WG) void k_sc_assemble_off(Dev d, const uint8_t* mask) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9LL * d.sc_noff) return;
  const int blk = (int)(t / 9), i = (int)(t - 9LL * blk);
  const int e0 = d.sc_coff[blk], e1 = d.sc_coff[blk + 1];
  if (e0 == e1) return;
  if (mask && !mask[d.slot_prob[d.sc_contrib[e0].z]]) return;
  real acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = 0.f;
  for (int e = e0; e < e1; ++e) {
    const int4 c = d.sc_contrib[e];
    const real* lmd = d.lmd + (size_t)c.z * LMD_STRIDE;
    const real sl[3] = {lmd[LMD_SL + 0], lmd[LMD_SL + 1], lmd[LMD_SL + 2]};
    real Hi[3][3];
    load_p(lmd, Hi);
    // row i of G_a
    const real ja0 = rec_float(d, c.x, i), ja1 = rec_float(d, c.x, 9 + i);
    real ga[3], tn[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) ga[m] = (ja0 * rec_float(d, c.x, 18 + m) + ja1 * rec_float(d, c.x, 21 + m)) * sl[m];
#pragma unroll
    for (int n = 0; n < 3; ++n) tn[n] = ga[0] * Hi[0][n] + ga[1] * Hi[1][n] + ga[2] * Hi[2][n];
    real Jb[2][9], Gb[9][3];
    sc_load_g(d, c.y, sl, Jb, Gb);
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] -= tn[0] * Gb[j][0] + tn[1] * Gb[j][1] + tn[2] * Gb[j][2];
  }
  real* out = d.scb + (size_t)blk * 81 + 9 * i;
#pragma unroll
  for (int j = 0; j < 9; ++j) out[j] = acc[j];
}

// Diagonal block of camera c, row i (one thread): sum over the camera's
// observations (camera order) of (J^T J - G H~^-1 G^T) row i.
__global__ __launch_bounds__(WG) void k_sc_assemble_diag(Dev d, const uint8_t* mask) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * d.NC) return;
  const int c = t / 9, i = t - 9 * c;
  if (mask && !mask[d.cam_prob[c]]) return;
  real acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = 0.f;
  for (int e = d.cam_obs_off[c]; e < d.cam_obs_off[c + 1]; ++e) {
    const int q = d.cam_obs_idx[e];
    const int slot = d.lm_slot[d.obs_lm[q]];
    const int ri = d.slot_zoff[slot] + (q - d.slot_obs0[slot]);
    const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
    const real sl[3] = {lmd[LMD_SL + 0], lmd[LMD_SL + 1], lmd[LMD_SL + 2]};
    real Hi[3][3], J[2][9], G[9][3];
    load_p(lmd, Hi);
    sc_load_g(d, ri, sl, J, G);
    real tn[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) tn[n] = G[i][0] * Hi[0][n] + G[i][1] * Hi[1][n] + G[i][2] * Hi[2][n];
#pragma unroll
    for (int j = 0; j < 9; ++j)
      acc[j] += J[0][i] * J[0][j] + J[1][i] * J[1][j] - (tn[0] * G[j][0] + tn[1] * G[j][1] + tn[2] * G[j][2]);
  }
  real* out = d.scb + (size_t)(d.sc_noff + c) * 81 + 9 * i;
#pragma unroll
  for (int j = 0; j < 9; ++j) out[j] = acc[j];
}

// Product with the assembled reduced matrix, one wavefront per camera row:
// vy_c = sum over the row's blocks of B (S v)_other (B^T for the transposed
// entries), lanes over blocks in a fixed order and a fixed reduction tree.
template <bool PCG>
__global__ __launch_bounds__(64) void k_sc_matvec(Dev d) {
  const int c = blockIdx.x, lane = threadIdx.x;
  const int prob = d.cam_prob[c];
  if (!d.active[prob] || (PCG && d.done[prob])) return;
  real acc[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) acc[a] = 0.f;
  for (int e = d.sc_rowoff[c] + lane; e < d.sc_rowoff[c + 1]; e += 64) {
    const int2 en = d.sc_rowent[e];
    const real* B = d.scb + (size_t)(en.x & 0x7fffffff) * 81;
    const real4* vs = reinterpret_cast<const real4*>(d.vzs) + 3 * (size_t)en.y;
    const real4 v0 = vs[0], v1 = vs[1], v2 = vs[2];
    const real v[9] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w, v2.x};
    if (en.x >= 0) {
#pragma unroll
      for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int j = 0; j < 9; ++j) acc[a] += B[9 * a + j] * v[j];
    } else {
#pragma unroll
      for (int a = 0; a < 9; ++a)
#pragma unroll
        for (int j = 0; j < 9; ++j) acc[a] += B[9 * j + a] * v[j];
    }
  }
#pragma unroll
  for (int a = 0; a < 9; ++a) acc[a] = wave_sum_f(acc[a]);
  if (lane < 9) {
    real s = acc[0];
#pragma unroll
    for (int a = 1; a < 9; ++a) s = (lane == a) ? acc[a] : s;
    d.vy[9 * c + lane] = s;
  }
}

// Back-substitution (eq. backsub_sc) per landmark: dl~ = -H~^-1 (b_l + (J_l S_l)^T J_p p'),
// p' = S dx_p, and the undamped model decrease -sum u (2 r + u), u = J_p p' + J_l S_l dl~.
template <int TEAM, int OPL>
__device__ __forceinline__ void sc_backsub(const Dev& d, int slot, int lane) {
  const int prob = d.slot_prob[slot];
  if (!d.active[prob]) return;
  const int lm = d.slot_lm[slot];
  const int k = d.slot_k[slot], r0 = d.slot_zoff[slot];
  const real* lmd = d.lmd + (size_t)slot * LMD_STRIDE;
  const real sl[3] = {lmd[LMD_SL + 0], lmd[LMD_SL + 1], lmd[LMD_SL + 2]};
  real u[OPL][2];
  real c[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    u[m][0] = u[m][1] = 0.f;
    if (o < k) {
      real J[2][9], Lu[2][3];
      load_rec(d, r0 + o, J, Lu);
      const int cam = 9 * d.rec_cam[r0 + o];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const real pa = d.s_cam[cam + a] * d.vx[cam + a];
        u[m][0] += J[0][a] * pa;
        u[m][1] += J[1][a] * pa;
      }
#pragma unroll
      for (int j = 0; j < 3; ++j) c[j] += (Lu[0][j] * u[m][0] + Lu[1][j] * u[m][1]) * sl[j];
    }
  }
  int buf = 0;
  team_sum_n<TEAM, 3>(c, nullptr, buf);
  real Hi[3][3];
  load_p(lmd, Hi);
  const real g[3] = {lmd[LMD_QR + 0] + c[0], lmd[LMD_QR + 1] + c[1], lmd[LMD_QR + 2] + c[2]};
  real dl[3];
#pragma unroll
  for (int n = 0; n < 3; ++n) dl[n] = -(Hi[n][0] * g[0] + Hi[n][1] * g[1] + Hi[n][2] * g[2]);
  real s2[1] = {0.f};
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = lane + TEAM * m;
    if (o < k) {
      real J[2][9], Lu[2][3];
      load_rec(d, r0 + o, J, Lu);
      const real4 rv = rec_plane(d, 6)[r0 + o];
      const real w0 = u[m][0] + Lu[0][0] * sl[0] * dl[0] + Lu[0][1] * sl[1] * dl[1] + Lu[0][2] * sl[2] * dl[2];
      const real w1 = u[m][1] + Lu[1][0] * sl[0] * dl[0] + Lu[1][1] * sl[1] * dl[1] + Lu[1][2] * sl[2] * dl[2];
      s2[0] += w0 * (2.f * rv.x + w0) + w1 * (2.f * rv.y + w1);
    }
  }
  team_sum_n<TEAM, 1>(s2, nullptr, buf);
  if (lane == 0) {
    d.dxl[3 * (size_t)lm + 0] = sl[0] * dl[0];
    d.dxl[3 * (size_t)lm + 1] = sl[1] * dl[1];
    d.dxl[3 * (size_t)lm + 2] = sl[2] * dl[2];
    d.lm_part[lm] = -(double)s2[0];
  }
}

struct ScBacksubF {
  const Dev& d;
  template <int TEAM, int OPL>
  __device__ __forceinline__ void run(int slot, int lane) const { sc_backsub<TEAM, OPL>(d, slot, lane); }
};

__global__ __launch_bounds__(WG) void k_sc_backsub(Dev d, ImplGrid m) { impl_dispatch(m, ScBacksubF{d}); }

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ----------------------------------------------------- launchers

// Launch description of classes 0..4 (in launch order 4, 3, 2, 1, 0); *n gets
// the number of workgroups.  With skip4, class 4 is left out.
static ClassGrid class_grid(const Launch& L, int* n, bool skip4 = false) {
  ClassGrid m;
  *n = 0;
  for (int j = 0; j < 5; ++j) {
    const WorkClass& c = L.wc[4 - j];
    const int per = mv_per_wg(j);
    m.nblk[j] = (j == 0 && skip4) ? 0 : (c.slots + per - 1) / per;
    m.first[j] = c.first_slot;
    m.end[j] = c.first_slot + c.slots;
    *n += m.nblk[j];
  }
  return m;
}

// Launch description of all six classes for the implicit kernels.
static ImplGrid impl_grid(const Launch& L, int* n) {
  ImplGrid m;
  *n = 0;
  for (int j = 0; j < 6; ++j) {
    const WorkClass& c = L.wc[5 - j];
    const int per = WG / impl_team(j);
    m.nblk[j] = (c.slots + per - 1) / per;
    m.first[j] = c.first_slot;
    m.end[j] = c.first_slot + c.slots;
    *n += m.nblk[j];
  }
  return m;
}

#define LAUNCH_CHECK()                       \
  do {                                       \
    hipError_t e_ = hipGetLastError();       \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

hipError_t launch_cam_linearize(const Dev& d, const Launch& L, bool jac, bool use_new, const uint8_t* mask) {
  if (d.NC == 0) return hipSuccess;
  const real* cam = use_new ? d.cam_new : d.cam;
  const real4* pts = use_new ? d.pts_new : d.pts;
  if (jac)
    hipLaunchKernelGGL(k_cam_linearize<true>, dim3(d.NC), dim3(64), 0, L.stream, d, cam, pts, mask);
  else
    hipLaunchKernelGGL(k_cam_linearize<false>, dim3(d.NC), dim3(64), 0, L.stream, d, cam, pts, mask);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_prob_sum(const Dev& d, const Launch& L, const double* vals, const int32_t* off, double* out,
                           const uint8_t* mask) {
  hipLaunchKernelGGL(k_prob_sum_chunks, dim3(d.P * d.sum_chunks), dim3(SUM_THREADS), 0, L.stream, vals, off, d.psum,
                     d.sum_chunks, mask);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_prob_sum_final, dim3(d.P), dim3(64), 0, L.stream, off, d.psum, d.sum_chunks, out, mask);
  LAUNCH_CHECK();
  return hipSuccess;
}

// Class 5 (few, long workgroups) runs on the side stream concurrently with
// classes 0..4 when both are present.
hipError_t launch_marginalize(const Dev& d, const Launch& L, const uint8_t* mask) {
  const WorkClass* w = L.wc;
  if (d.sc) {  // explicit Schur complement: normal-equation terms per landmark
    int n = 0;
    const ImplGrid m = impl_grid(L, &n);
    if (n) hipLaunchKernelGGL(k_sc_prepare, dim3(n), dim3(WG), 0, L.stream, d, m, mask);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  int n = 0;
  const ClassGrid m = class_grid(L, &n);
  const bool side = w[5].slots && n && L.side && L.fork && L.join;
  if (side) {
    hipError_t e = hipEventRecord(L.fork, L.stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(L.side, L.fork, 0);
    if (e != hipSuccess) return e;
  }
  if (w[5].slots) {
    if (d.implicit)
      hipLaunchKernelGGL(k_marginalize_huge<true>, dim3(w[5].slots), dim3(WG), 0, side ? L.side : L.stream, d,
                         w[5].first_slot, mask);
    else
      hipLaunchKernelGGL(k_marginalize_chunks, dim3(L.qjobs), dim3(WG), 0, side ? L.side : L.stream, d, mask);
  }
  LAUNCH_CHECK();
  if (n) {
    if (d.implicit)
      hipLaunchKernelGGL(k_marginalize<true>, dim3(n), dim3(WG), 0, L.stream, d, m, mask);
    else
      hipLaunchKernelGGL(k_marginalize<false>, dim3(n), dim3(WG), 0, L.stream, d, m, mask);
  }
  LAUNCH_CHECK();
  if (side) {
    hipError_t e = hipEventRecord(L.join, L.side);
    if (e == hipSuccess) e = hipStreamWaitEvent(L.stream, L.join, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The landmarks of class 5 (k > 113: few, each a long stream for one workgroup)
// run on the side stream concurrently with the other classes, forked from and
// joined back into the context stream by events; without a side stream they
// run first on the context stream.
static hipError_t side_fork(const Launch& L, bool side) {
  if (!side) return hipSuccess;
  hipError_t e = hipEventRecord(L.fork, L.stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(L.side, L.fork, 0);
  return e;
}

static hipError_t side_join(const Launch& L, bool side) {
  if (!side) return hipSuccess;
  hipError_t e = hipEventRecord(L.join, L.side);
  if (e == hipSuccess) e = hipStreamWaitEvent(L.stream, L.join, 0);
  return e;
}

hipError_t launch_damp(const Dev& d, const Launch& L, const uint8_t* mask) {
  const WorkClass* w = L.wc;
  if (d.sc) {  // (H_ll + lambda I)^-1, then the reduced matrix assembled anew
    if (d.NS) hipLaunchKernelGGL(k_sc_damp, dim3(nblocks(d.NS, WG)), dim3(WG), 0, L.stream, d, mask);
    LAUNCH_CHECK();
    if (d.sc_noff)
      hipLaunchKernelGGL(k_sc_assemble_off, dim3(nblocks(9LL * d.sc_noff, WG)), dim3(WG), 0, L.stream, d, mask);
    LAUNCH_CHECK();
    if (d.NC) hipLaunchKernelGGL(k_sc_assemble_diag, dim3(nblocks(9LL * d.NC, WG)), dim3(WG), 0, L.stream, d, mask);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  if (d.implicit) {
    if (d.NS) hipLaunchKernelGGL(k_damp_implicit, dim3(nblocks(d.NS, WG)), dim3(WG), 0, L.stream, d, mask);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  int n = 0;
  const ClassGrid m = class_grid(L, &n);
  const bool side = w[5].slots && n && L.side && L.fork && L.join;
  hipError_t e = side_fork(L, side);
  if (e != hipSuccess) return e;
  if (w[5].slots)
    hipLaunchKernelGGL(k_damp_huge, dim3(w[5].slots), dim3(WG), 0, side ? L.side : L.stream, d, w[5].first_slot,
                       mask);
  LAUNCH_CHECK();
  if (n) hipLaunchKernelGGL(k_damp, dim3(n), dim3(WG), 0, L.stream, d, m, mask);
  LAUNCH_CHECK();
  e = side_join(L, side);
  if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_precond_rhs(const Dev& d, const Launch& L) {
  if (d.sc) {
    if (d.NO) hipLaunchKernelGGL(k_sc_precond_obs, dim3(nblocks(d.NO, WG)), dim3(WG), 0, L.stream, d);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_precond_cam, dim3(d.NC), dim3(64), 0, L.stream, d);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  if (d.implicit) {
    if (d.NO) hipLaunchKernelGGL(k_precond_obs_implicit, dim3(nblocks(d.NO, WG)), dim3(WG), 0, L.stream, d);
    LAUNCH_CHECK();
    hipLaunchKernelGGL(k_precond_cam, dim3(d.NC), dim3(64), 0, L.stream, d);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  // explicit blocks: the per-observation records come from the damping
  hipLaunchKernelGGL(k_precond_cam, dim3(d.NC), dim3(64), 0, L.stream, d);
  LAUNCH_CHECK();
  return hipSuccess;
}

// The landmarks with k > 113 (few, each a long stream for one workgroup) run
// on a side stream concurrently with the main product, forked from and joined
// back into the context stream by events (also inside captured graphs).
// Product over all landmark blocks: the class-5 row blocks (on the side
// stream, concurrently with the rest, when huge_side), class 4 (inside the
// main launch, or on its own when large_sep), classes 0..3, then the sum of
// the class-5 partials.  The launch shapes are the tunables of Launch.
template <bool PCG, bool LARGE, int RBS, bool NT>
static void launch_small3(const Dev& d, const Launch& L, const ClassGrid& m, int n, const real* v) {
  if (L.persist > 0 && n > L.persist)
    hipLaunchKernelGGL((k_matvec<PCG, LARGE, RBS, true, NT>), dim3(L.persist), dim3(WG), 0, L.stream, d, m, n, v);
  else
    hipLaunchKernelGGL((k_matvec<PCG, LARGE, RBS, false, NT>), dim3(n), dim3(WG), 0, L.stream, d, m, n, v);
}

// Launch::nt bit 1: non-temporal loads of the blocks of classes 0..3.
template <bool PCG, bool LARGE>
static void launch_small(const Dev& d, const Launch& L, const ClassGrid& m, int n, const real* v) {
  const bool nt = (L.nt & 2) != 0;
  if (L.mv_rbs == 0) {
    if (nt)
      launch_small3<PCG, LARGE, 0, true>(d, L, m, n, v);
    else
      launch_small3<PCG, LARGE, 0, false>(d, L, m, n, v);
  } else {
    if (nt)
      launch_small3<PCG, LARGE, 1, true>(d, L, m, n, v);
    else
      launch_small3<PCG, LARGE, 1, false>(d, L, m, n, v);
  }
}

// Product over all landmark blocks.  Slots are ordered by decreasing k, so the
// landmarks with k >= 29 form the prefix [0, n45); its first rows_n slots (k at
// least the tuned edge) go to the row-block kernel (on the side stream when
// huge_side), the rest of the prefix to the large-landmark path (inside the
// main launch, or on its own when large_sep), then classes 0..3, then the sum
// of the row-block partials.
template <bool PCG>
static hipError_t launch_matvec(const Dev& d, const Launch& L, const real* v) {
  // every form gathers S v from vzs: in PCG the PCG kernels keep vzs = S z;
  // otherwise it is formed from v here (v == nullptr: already formed)
  if (!PCG && v && d.NC) {
    hipLaunchKernelGGL(k_prescale, dim3(nblocks(9 * d.NC, WG)), dim3(WG), 0, L.stream, d, v);
    LAUNCH_CHECK();
  }
  if (d.sc) {  // product with the assembled reduced matrix into vy
    if (d.NC) hipLaunchKernelGGL(k_sc_matvec<PCG>, dim3(d.NC), dim3(64), 0, L.stream, d);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  if (d.implicit) {
    int n = 0;
    const ImplGrid m = impl_grid(L, &n);
    if (n) hipLaunchKernelGGL(k_matvec_implicit<PCG>, dim3(n), dim3(WG), 0, L.stream, d, m);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  v = d.vzs;
  const bool rows = L.rows_n > 0 && L.hjobs > 0;
  const bool side = rows && L.huge_side && L.side && L.fork && L.join;
  const hipStream_t hs = side ? L.side : L.stream;
  if (rows) {
    if (side) {
      hipError_t e = hipEventRecord(L.fork, L.stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(L.side, L.fork, 0);
      if (e != hipSuccess) return e;
    }
    if (L.nt & 1)
      hipLaunchKernelGGL((k_matvec_rows<PCG, true>), dim3(L.hjobs), dim3(WG), 0, hs, d, 0, L.huge_rows, v);
    else
      hipLaunchKernelGGL((k_matvec_rows<PCG, false>), dim3(L.hjobs), dim3(WG), 0, hs, d, 0, L.huge_rows, v);
    LAUNCH_CHECK();
    if (L.huge_rows < 2 * class_kmax(5))
      hipLaunchKernelGGL(k_matvec_combine<PCG>, dim3(L.rows_n), dim3(WG), 0, hs, d, 0, L.huge_rows);
    LAUNCH_CHECK();
  }
  const int nlarge = L.n45 - L.rows_n;
  const bool sep = L.large_sep && nlarge > 0;
  if (sep) {
    if (L.nt & 1)
      hipLaunchKernelGGL((k_matvec_large<PCG, true>), dim3(nlarge), dim3(WG), 0, L.stream, d, L.rows_n, v);
    else
      hipLaunchKernelGGL((k_matvec_large<PCG, false>), dim3(nlarge), dim3(WG), 0, L.stream, d, L.rows_n, v);
    LAUNCH_CHECK();
  }
  int n = 0;
  ClassGrid m = class_grid(L, &n, true);
  if (!sep && nlarge > 0) {  // the large-landmark path inside the main launch
    m.nblk[0] = nlarge;
    m.first[0] = L.rows_n;
    m.end[0] = L.n45;
    n += nlarge;
  }
  if (n) {
    if (m.nblk[0])
      launch_small<PCG, true>(d, L, m, n, v);
    else
      launch_small<PCG, false>(d, L, m, n, v);
    LAUNCH_CHECK();
  }
  if (side) {
    hipError_t e = hipEventRecord(L.join, L.side);
    if (e == hipSuccess) e = hipStreamWaitEvent(L.stream, L.join, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pcg_init(const Dev& d, const Launch& L) {
  hipLaunchKernelGGL(k_pcg_init, dim3(nblocks(d.NC > 0 ? d.NC : 1, WG)), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_pcg_init_scalars, dim3(nblocks(d.P > 0 ? d.P : 1, WG / 64)), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  if (d.test_sep && d.P > 0) hipLaunchKernelGGL(k_pcg_test, dim3(nblocks(d.P, WG / 64)), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_matvec(const Dev& d, const Launch& L) { return launch_matvec<true>(d, L, nullptr); }

hipError_t launch_pcg_vector(const Dev& d, const Launch& L) {
  hipLaunchKernelGGL(k_pcg_q, dim3(d.NC), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  hipLaunchKernelGGL(k_pcg_update, dim3(nblocks(d.NC, UPD_CAMS)), dim3(UPD_THREADS), 0, L.stream, d);
  LAUNCH_CHECK();
  if (d.test_sep && d.P > 0) hipLaunchKernelGGL(k_pcg_test, dim3(nblocks(d.P, WG / 64)), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_pcg_final(const Dev& d, const Launch& L) {
  hipLaunchKernelGGL(k_pcg_final, dim3(1), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_pcg_iteration(const Dev& d, const Launch& L) {
  hipError_t e = launch_matvec(d, L);
  if (e != hipSuccess) return e;
  return launch_pcg_vector(d, L);
}

hipError_t launch_backsub(const Dev& d, const Launch& L) {
  const WorkClass* w = L.wc;
  if (d.sc) {
    int n = 0;
    const ImplGrid m = impl_grid(L, &n);
    if (n) hipLaunchKernelGGL(k_sc_backsub, dim3(n), dim3(WG), 0, L.stream, d, m);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  if (d.implicit) {
    int n = 0;
    const ImplGrid m = impl_grid(L, &n);
    if (n) hipLaunchKernelGGL(k_backsub_implicit, dim3(n), dim3(WG), 0, L.stream, d, m);
    LAUNCH_CHECK();
    return hipSuccess;
  }
  // the landmark kernels gather S dx_p from vzs
  if (d.NC) hipLaunchKernelGGL(k_prescale, dim3(nblocks(9 * d.NC, WG)), dim3(WG), 0, L.stream, d, d.vx);
  LAUNCH_CHECK();
  int n = 0;
  const ClassGrid m = class_grid(L, &n);
  const bool side = w[5].slots && n && L.side && L.fork && L.join;
  hipError_t e = side_fork(L, side);
  if (e != hipSuccess) return e;
  if (w[5].slots)
    hipLaunchKernelGGL(k_backsub_huge, dim3(w[5].slots), dim3(WG), 0, side ? L.side : L.stream, d, w[5].first_slot);
  LAUNCH_CHECK();
  if (n) hipLaunchKernelGGL(k_backsub, dim3(n), dim3(WG), 0, L.stream, d, m);
  LAUNCH_CHECK();
  return side_join(L, side);
}

hipError_t launch_update(const Dev& d, const Launch& L) {
  const long long n = d.NC > d.NL ? d.NC : d.NL;
  hipLaunchKernelGGL(k_update, dim3(nblocks(n, WG)), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_commit(const Dev& d, const Launch& L) {
  const long long n = d.NC > d.NL ? d.NC : d.NL;
  hipLaunchKernelGGL(k_commit, dim3(nblocks(n, WG)), dim3(WG), 0, L.stream, d);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_matvec_timing(const Dev& d, const Launch& L) { return launch_matvec<false>(d, L, nullptr); }

hipError_t launch_prescale_z(const Dev& d, const Launch& L) {
  if (d.NC) hipLaunchKernelGGL(k_prescale, dim3(nblocks(9 * d.NC, WG)), dim3(WG), 0, L.stream, d, d.vz);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_matvec_only(const Dev& d, const Launch& L, const real* v_scaled, real* out) {
  hipError_t e = launch_matvec<false>(d, L, v_scaled);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cam_gather_product, dim3(d.NC), dim3(64), 0, L.stream, d, v_scaled, out);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_debug_linearization(const Dev& d, const Launch& L, real* r, real* Jp, real* Jl) {
  if (d.NO == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_lin, dim3(nblocks(d.NO, WG)), dim3(WG), 0, L.stream, d, r, Jp, Jl);
  LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace sqrtba
