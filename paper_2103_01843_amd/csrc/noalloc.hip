// The reduced-camera-system product without allocation: the scratch of the
// product kernels (the scaled input vector, per-observation outputs and
// row-block partials) lives in a
// file-scope device array instead of the context's workspace, so the entry
// point that uses it (sqrtba_rcs_matvec_noalloc) calls no allocator and can be
// used under HIP graph capture or in loops that must not allocate.
//
// The array exists once per device that the library runs on and lives until
// the process ends.  Its device address is looked up once per device, with
// that device current, and kept; host code passes that address, never the
// array's name, to kernels.
#include <mutex>

#include "device.h"

namespace sqrtba {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Zero n elements (a fill kernel rather than a memset node, which graph
// capture records badly).
__global__ __launch_bounds__(256) void k_zero(real4* p, int64_t n4) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_real4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

int64_t noalloc_out_elems(int64_t out_elems) { return (out_elems + 63) & ~int64_t(63); }

int64_t noalloc_elems(int64_t n_cams, int64_t out_elems, int64_t partial_elems) {
  return noalloc_out_elems(12 * n_cams) + noalloc_out_elems(out_elems) + partial_elems;
}

hipError_t launch_matvec_noalloc(const Dev& d, const Launch& L, void* scratch_ptr, int64_t out_elems,
                                 const real* v, real* out) {
  Dev s = d;
  s.vzs = static_cast<real*>(scratch_ptr);  // pads are never read
  s.obsbuf = s.vzs + noalloc_out_elems(12 * (int64_t)d.NC);
  s.zpart = s.obsbuf + noalloc_out_elems(out_elems);
  // the outputs of problems the product skips (inactive ones) read as zero, not
  // as what the previous call left in the shared array
  const int64_t n4 = noalloc_out_elems(out_elems) / 4;
  if (n4 > 0) {
    const int blocks = (int)((n4 + 255) / 256 < 4096 ? (n4 + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, L.stream, reinterpret_cast<real4*>(s.obsbuf), n4);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_matvec_only(s, L, v, out);
}

}  // namespace sqrtba
