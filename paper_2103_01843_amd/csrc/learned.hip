// Learned correction of the block-Jacobi preconditioner (not part of the
// paper; the project's own extension).  Per camera, a small MLP
// (64 -> 128 -> 128 -> 81, tanh, bfloat16 weights, FP32 accumulation) reads
// features of the damped 9x9 block P = L L^T and emits E; the inverse block is
//     M^-1 = C C^T,  C = L^-T T,  T = I + alpha tanh(tril(E)),  alpha = 0.1,
// symmetric positive definite by construction (diag(T) >= 0.9) and equal to
// plain block-Jacobi for E = 0.  Training minimizes, over pairs (p, q = A p)
// traced from the solver's own PCG runs, the mean of |M^-1 q_i - p_i|^2 / |p_i|^2
// per camera i, with hand-written forward, backward and Adam kernels.

#include <hip/hip_runtime.h>

#include "learned.h"

namespace sqrtba {

namespace {

constexpr int NIN = MLP_IN, NH = MLP_HIDDEN, NOUT = MLP_OUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NOUT, NPAR = OFF_B3 + NOUT;
static_assert(NPAR == MLP_PARAMS, "parameter layout");
constexpr float ALPHA = 0.1f;
constexpr int TILE = 16;  // samples per workgroup in training
constexpr int TPB = 256;

__device__ __forceinline__ float bf(const uint16_t* w, int i) {
  return __uint_as_float(((uint32_t)w[i]) << 16);
}

__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// out[s][j] = act(b[j] + sum_i in[s][i] W[i][j]) for s < S, by the whole workgroup
template <bool TANH>
__device__ __forceinline__ void dense(const float* in, int nin, float* out, int nout, const uint16_t* W, int w0, int b0,
                                      int S) {
  for (int idx = threadIdx.x; idx < S * nout; idx += blockDim.x) {
    const int s = idx / nout, j = idx - s * nout;
    float acc = bf(W, b0 + j);
    const float* x = in + s * nin;
    for (int i = 0; i < nin; ++i) acc += x[i] * bf(W, w0 + i * nout + j);
    out[idx] = TANH ? tanhf(acc) : acc;
  }
}

// Unpack the lower Cholesky factor (packed row-major lower triangle, 45 floats).
__device__ __forceinline__ void unpack_L(const float* Lp, float (*L)[9]) {
  int e = 0;
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int b = 0; b < 9; ++b) L[a][b] = (b <= a) ? Lp[e++] : 0.f;
}

// C = L^-T T: solve L^T C = T column by column (back substitution).
__device__ __forceinline__ void factor_C(const float (*L)[9], const float (*T)[9], float (*Cm)[9]) {
#pragma unroll
  for (int col = 0; col < 9; ++col) {
#pragma unroll
    for (int a = 8; a >= 0; --a) {
      float v = T[a][col];
#pragma unroll
      for (int q = a + 1; q < 9; ++q) v -= L[q][a] * Cm[q][col];
      Cm[a][col] = v / L[a][a];
    }
  }
}

__device__ __forceinline__ void make_T(const float* e, float (*T)[9], float (*th)[9]) {
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int b = 0; b < 9; ++b) {
      th[a][b] = (b <= a) ? tanhf(e[9 * a + b]) : 0.f;
      T[a][b] = (a == b ? 1.f : 0.f) + ALPHA * th[a][b];
    }
}

// ---------------------------------------------------------------- inference

// One workgroup per tile of TILE cameras: features -> MLP -> M^-1 = C C^T into minv.
__global__ __launch_bounds__(TPB) void k_mlp_precond(Dev d, LearnDev m) {
  __shared__ float x[TILE * NIN];
  __shared__ float h1[TILE * NH];
  __shared__ float h2[TILE * NH];
  __shared__ float eo[TILE * NOUT];
  __shared__ float mats[TILE][4][81];  // per-sample 9x9 work matrices
  const int c0 = blockIdx.x * TILE;
  const int S = min(TILE, d.NC - c0);
  for (int idx = threadIdx.x; idx < S * NIN; idx += blockDim.x) x[idx] = m.feats[(size_t)c0 * NIN + idx];
  __syncthreads();
  dense<true>(x, NIN, h1, NH, m.wbf, OFF_W1, OFF_B1, S);
  __syncthreads();
  dense<true>(h1, NH, h2, NH, m.wbf, OFF_W2, OFF_B2, S);
  __syncthreads();
  dense<false>(h2, NH, eo, NOUT, m.wbf, OFF_W3, OFF_B3, S);
  __syncthreads();
  if ((int)threadIdx.x < S) {
    const int c = c0 + threadIdx.x;
    if (!d.active[d.cam_prob[c]]) return;
    float(*L)[9] = reinterpret_cast<float(*)[9]>(mats[threadIdx.x][0]);
    float(*T)[9] = reinterpret_cast<float(*)[9]>(mats[threadIdx.x][1]);
    float(*th)[9] = reinterpret_cast<float(*)[9]>(mats[threadIdx.x][2]);
    float(*Cm)[9] = reinterpret_cast<float(*)[9]>(mats[threadIdx.x][3]);
    unpack_L(m.lfac + 45 * (size_t)c, L);
    make_T(eo + NOUT * threadIdx.x, T, th);
    factor_C(L, T, Cm);
    real* mi = d.minv + 81 * (size_t)c;
#pragma unroll
    for (int a = 0; a < 9; ++a)
#pragma unroll
      for (int b = 0; b < 9; ++b) {
        float v = 0.f;
#pragma unroll
        for (int q = 0; q < 9; ++q) v += Cm[a][q] * Cm[b][q];
        mi[9 * a + b] = v;
      }
  }
}

// ---------------------------------------------------------------- training

// One workgroup per tile of TILE samples: forward, per-sample loss and dE,
// backward, and this tile's share of the weight gradient (written to
// part[blockIdx.x][0..NPAR)) and of the loss (loss_part[blockIdx.x]).  Samples
// come either from the trace store (sample list of (record, camera)) or from
// explicit arrays (feats, lfac, p, q of n samples).  scale = 1 / batch size.
__global__ __launch_bounds__(TPB) void k_mlp_grad(LearnDev m, SampleSrc src, int n, float scale, float* part,
                                                  double* loss_part) {
  __shared__ float x[TILE * NIN];
  __shared__ float h1[TILE * NH];
  __shared__ float h2[TILE * NH];
  __shared__ float dE[TILE * NOUT];
  __shared__ float d2[TILE * NH];
  __shared__ float d1[TILE * NH];
  __shared__ float lsum[TILE];
  __shared__ float mats[TILE][4][81];  // per-sample 9x9 work matrices
  const int s0 = blockIdx.x * TILE;
  const int S = min(TILE, n - s0);
  // gather inputs
  for (int idx = threadIdx.x; idx < S * NIN; idx += blockDim.x) {
    const int s = idx / NIN, i = idx - s * NIN;
    x[idx] = src.feat(s0 + s)[i];
  }
  __syncthreads();
  dense<true>(x, NIN, h1, NH, m.wbf, OFF_W1, OFF_B1, S);
  __syncthreads();
  dense<true>(h1, NH, h2, NH, m.wbf, OFF_W2, OFF_B2, S);
  __syncthreads();
  dense<false>(h2, NH, dE, NOUT, m.wbf, OFF_W3, OFF_B3, S);  // dE holds e for now
  __syncthreads();
  if ((int)threadIdx.x < TILE) {
    const int s = threadIdx.x;
    float l = 0.f;
    float g_E[81];
#pragma unroll
    for (int e = 0; e < 81; ++e) g_E[e] = 0.f;
    if (s < S) {
      const float* p = src.p(s0 + s);
      const float* q = src.q(s0 + s);
      float pp = 0.f;
#pragma unroll
      for (int a = 0; a < 9; ++a) pp += p[a] * p[a];
      if (pp > 0.f) {
        float(*L)[9] = reinterpret_cast<float(*)[9]>(mats[s][0]);
        float(*T)[9] = reinterpret_cast<float(*)[9]>(mats[s][1]);
        float(*th)[9] = reinterpret_cast<float(*)[9]>(mats[s][2]);
        float(*Cm)[9] = reinterpret_cast<float(*)[9]>(mats[s][3]);
        unpack_L(src.lfac(s0 + s), L);
        make_T(dE + NOUT * s, T, th);
        factor_C(L, T, Cm);
        float u[9], mm[9], r[9], gm[9], gu[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {  // u = C^T q
          float v = 0.f;
#pragma unroll
          for (int b = 0; b < 9; ++b) v += Cm[b][a] * q[b];
          u[a] = v;
        }
#pragma unroll
        for (int a = 0; a < 9; ++a) {  // m = C u, r = m - p
          float v = 0.f;
#pragma unroll
          for (int b = 0; b < 9; ++b) v += Cm[a][b] * u[b];
          mm[a] = v;
          r[a] = v - p[a];
          l += r[a] * r[a];
        }
        l /= pp;
#pragma unroll
        for (int a = 0; a < 9; ++a) gm[a] = 2.f * scale * r[a] / pp;
#pragma unroll
        for (int b = 0; b < 9; ++b) {  // gu = C^T gm
          float v = 0.f;
#pragma unroll
          for (int a = 0; a < 9; ++a) v += Cm[a][b] * gm[a];
          gu[b] = v;
        }
        // g_C = gm u^T + q gu^T;  g_T = L^-1 g_C (forward substitution per column),
        // stored over T, which is no longer needed
        float(*gT)[9] = T;
#pragma unroll
        for (int col = 0; col < 9; ++col) {
#pragma unroll
          for (int a = 0; a < 9; ++a) {
            float v = gm[a] * u[col] + q[a] * gu[col];
#pragma unroll
            for (int b = 0; b < a; ++b) v -= L[a][b] * gT[b][col];
            gT[a][col] = v / L[a][a];
          }
        }
#pragma unroll
        for (int a = 0; a < 9; ++a)
#pragma unroll
          for (int b = 0; b <= a; ++b) g_E[9 * a + b] = gT[a][b] * ALPHA * (1.f - th[a][b] * th[a][b]);
        (void)mm;
      }
    }
    lsum[s] = l;
#pragma unroll
    for (int e = 0; e < 81; ++e) dE[NOUT * s + e] = (s < S) ? g_E[e] : 0.f;
  }
  __syncthreads();
  // backward through the layers (rows s >= S of dE are zero)
  for (int idx = threadIdx.x; idx < TILE * NH; idx += blockDim.x) {
    const int s = idx / NH, j = idx - s * NH;
    float acc = 0.f;
    if (s < S) {
      for (int e = 0; e < NOUT; ++e) acc += dE[NOUT * s + e] * bf(m.wbf, OFF_W3 + j * NOUT + e);
      acc *= 1.f - h2[idx] * h2[idx];
    }
    d2[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < TILE * NH; idx += blockDim.x) {
    const int s = idx / NH, i = idx - s * NH;
    float acc = 0.f;
    if (s < S) {
      for (int j = 0; j < NH; ++j) acc += d2[NH * s + j] * bf(m.wbf, OFF_W2 + i * NH + j);
      acc *= 1.f - h1[idx] * h1[idx];
    }
    d1[idx] = acc;
  }
  __syncthreads();
  float* g = part + (size_t)blockIdx.x * NPAR;
  for (int idx = threadIdx.x; idx < NPAR; idx += blockDim.x) {
    float acc = 0.f;
    if (idx < OFF_B1) {
      const int i = idx / NH, j = idx - i * NH;
      for (int s = 0; s < S; ++s) acc += x[NIN * s + i] * d1[NH * s + j];
    } else if (idx < OFF_W2) {
      const int j = idx - OFF_B1;
      for (int s = 0; s < S; ++s) acc += d1[NH * s + j];
    } else if (idx < OFF_B2) {
      const int t = idx - OFF_W2, i = t / NH, j = t - i * NH;
      for (int s = 0; s < S; ++s) acc += h1[NH * s + i] * d2[NH * s + j];
    } else if (idx < OFF_W3) {
      const int j = idx - OFF_B2;
      for (int s = 0; s < S; ++s) acc += d2[NH * s + j];
    } else if (idx < OFF_B3) {
      const int t = idx - OFF_W3, j = t / NOUT, e = t - j * NOUT;
      for (int s = 0; s < S; ++s) acc += h2[NH * s + j] * dE[NOUT * s + e];
    } else {
      const int e = idx - OFF_B3;
      for (int s = 0; s < S; ++s) acc += dE[NOUT * s + e];
    }
    g[idx] = acc;
  }
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += (double)lsum[s];
    loss_part[blockIdx.x] = t;
  }
}

// grad[i] = sum over tiles of part[t][i] (fixed order)
__global__ __launch_bounds__(TPB) void k_grad_reduce(const float* part, int tiles, float* grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPAR) return;
  float s = 0.f;
  for (int t = 0; t < tiles; ++t) s += part[(size_t)t * NPAR + i];
  grad[i] = s;
}

// Adam on the FP32 master weights, then the bfloat16 copy used by the kernels.
__global__ __launch_bounds__(TPB) void k_adam(LearnDev m, const float* grad, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPAR) return;
  const float g = grad[i];
  const float mo = b1 * m.adam_m[i] + (1.f - b1) * g;
  const float vo = b2 * m.adam_v[i] + (1.f - b2) * g * g;
  m.adam_m[i] = mo;
  m.adam_v[i] = vo;
  const float w = m.w32[i] - lr * (mo / c1) / (sqrtf(vo / c2) + eps);
  m.w32[i] = w;
  m.wbf[i] = to_bf16(w);
}

__global__ __launch_bounds__(TPB) void k_to_bf16(LearnDev m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NPAR) m.wbf[i] = to_bf16(m.w32[i]);
}

}  // namespace

hipError_t launch_mlp_precond(const Dev& d, const LearnDev& m, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_precond, dim3((d.NC + TILE - 1) / TILE), dim3(TPB), 0, st, d, m);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const LearnDev& m, const SampleSrc& src, int n, float* part, double* loss_part,
                           float* grad, hipStream_t st) {
  const int tiles = (n + TILE - 1) / TILE;
  hipLaunchKernelGGL(k_mlp_grad, dim3(tiles), dim3(TPB), 0, st, m, src, n, 1.0f / (float)n, part, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_grad_reduce, dim3((NPAR + TPB - 1) / TPB), dim3(TPB), 0, st, part, tiles, grad);
  return hipGetLastError();
}

hipError_t launch_adam(const LearnDev& m, const float* grad, float lr, int step, hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((NPAR + TPB - 1) / TPB), dim3(TPB), 0, st, m, grad, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const LearnDev& m, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3((NPAR + TPB - 1) / TPB), dim3(TPB), 0, st, m);
  return hipGetLastError();
}

int mlp_tiles(int n) { return (n + TILE - 1) / TILE; }

}  // namespace sqrtba
