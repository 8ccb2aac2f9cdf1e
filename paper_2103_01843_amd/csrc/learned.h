// Internal interface of the learned block preconditioner (learned.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace sqrtba {

enum { MLP_IN = 64, MLP_HIDDEN = 128, MLP_OUT = 81, LFAC = 45 };
enum { MLP_PARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_OUT +
                    MLP_OUT };

// Network state on the device.
struct LearnDev {
  float* w32;       // FP32 master parameters (W1, b1, W2, b2, W3, b3; row-major [in][out])
  uint16_t* wbf;    // bfloat16 copy used by the kernels
  float* adam_m;
  float* adam_v;
  const float* feats;  // per camera: MLP_IN features of the current solve
  const float* lfac;   // per camera: lower Cholesky factor of the damped block (45, packed rows)
};

// Training samples: explicit arrays (mode 0) or (record, camera) pairs into the trace store (mode 1).
struct SampleSrc {
  int mode;
  int NC;
  const float* a_feat;   // mode 0: [n][64]
  const float* a_lfac;   //         [n][45]
  const float* a_p;      //         [n][9]
  const float* a_q;      //         [n][9]
  const int32_t* rec;    // mode 1: per sample, trace record
  const int32_t* cam;    //         per sample, camera
  const int32_t* rec_solve;  // record -> traced solve
  const float* t_feat;   // [solve][NC][64]
  const float* t_lfac;   // [solve][NC][45]
  const float* t_p;      // [record][NC][9]
  const float* t_q;      // [record][NC][9]
  __device__ const float* feat(int s) const {
    return mode == 0 ? a_feat + (size_t)MLP_IN * s
                     : t_feat + ((size_t)rec_solve[rec[s]] * NC + cam[s]) * MLP_IN;
  }
  __device__ const float* lfac(int s) const {
    return mode == 0 ? a_lfac + (size_t)LFAC * s : t_lfac + ((size_t)rec_solve[rec[s]] * NC + cam[s]) * LFAC;
  }
  __device__ const float* p(int s) const {
    return mode == 0 ? a_p + 9 * (size_t)s : t_p + ((size_t)rec[s] * NC + cam[s]) * 9;
  }
  __device__ const float* q(int s) const {
    return mode == 0 ? a_q + 9 * (size_t)s : t_q + ((size_t)rec[s] * NC + cam[s]) * 9;
  }
};

hipError_t launch_mlp_precond(const Dev& d, const LearnDev& m, hipStream_t st);
hipError_t launch_mlp_grad(const LearnDev& m, const SampleSrc& src, int n, float* part, double* loss_part,
                           float* grad, hipStream_t st);
hipError_t launch_adam(const LearnDev& m, const float* grad, float lr, int step, hipStream_t st);
hipError_t launch_to_bf16(const LearnDev& m, hipStream_t st);
int mlp_tiles(int n);

}  // namespace sqrtba
