// The C ABI's host code end to end under AddressSanitizer and UndefinedBehaviorSanitizer
// (CPU only): context creation, bookkeeping, upload, the launch-shape autotuner (graph
// capture of products), the stages one by one and the whole LM loop (deferred readbacks
// through the pinned staging slices, the PCG chunk loop and its flags), in both places
// of the PCG convergence test, on a single problem and on a batch.  The HIP runtime is
// replaced by a host stand-in (device memory is host memory, copies are memcpy, events,
// streams and graphs are tokens) and every kernel launcher is a no-op, so the device
// values the host reads are the zeros of the cleared workspace: the numbers mean
// nothing, the host code's memory accesses are what is checked.
#include "../../paper_2103_01843_amd/csrc/api.cpp"

#include <cstdlib>

// ---- host stand-in of the HIP runtime calls the library makes
namespace {
struct Token {
  int kind;
};
hipError_t token(void** out, int kind) {
  *out = new Token{kind};
  return hipSuccess;
}
}  // namespace

extern "C" {
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned int) {
  *d = h;
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  if (n) std::memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { return token(reinterpret_cast<void**>(s), 1); }
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<Token*>(s);
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return token(reinterpret_cast<void**>(e), 2); }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return token(reinterpret_cast<void**>(e), 2); }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<Token*>(e);
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { return token(reinterpret_cast<void**>(g), 3); }
hipError_t hipGraphInstantiate(hipGraphExec_t* ge, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return token(reinterpret_cast<void**>(ge), 4);
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t ge) {
  delete reinterpret_cast<Token*>(ge);
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete reinterpret_cast<Token*>(g);
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "host stand-in"; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
}  // extern "C"

// ---- every kernel launcher of the library is a no-op
namespace sqrtba {
hipError_t launch_cam_linearize(const Dev&, const Launch&, bool, bool, const uint8_t*) { return hipSuccess; }
hipError_t launch_prob_sum(const Dev&, const Launch&, const double*, const int32_t*, double*, const uint8_t*) {
  return hipSuccess;
}
hipError_t launch_marginalize(const Dev&, const Launch&, const uint8_t*) { return hipSuccess; }
hipError_t launch_damp(const Dev&, const Launch&, const uint8_t*) { return hipSuccess; }
hipError_t launch_precond_rhs(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_pcg_init(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_pcg_iteration(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_matvec(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_pcg_vector(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_pcg_final(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_backsub(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_update(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_commit(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_matvec_only(const Dev&, const Launch&, const real*, real*) { return hipSuccess; }
hipError_t launch_matvec_timing(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_prescale_z(const Dev&, const Launch&) { return hipSuccess; }
hipError_t launch_debug_linearization(const Dev&, const Launch&, real*, real*, real*) { return hipSuccess; }
hipError_t noalloc_scratch(int, void** out) {
  static unsigned char array[64];  // never dereferenced: no product runs here
  *out = array;
  return hipSuccess;
}
int64_t noalloc_out_elems(int64_t out_elems) { return out_elems; }
int64_t noalloc_elems(int64_t n_cams, int64_t out_elems, int64_t partial_elems) {
  return 12 * n_cams + out_elems + partial_elems;
}
hipError_t launch_matvec_noalloc(const Dev&, const Launch&, void*, int64_t, const real*, real*) { return hipSuccess; }
#ifndef SQRTBA_FP64
hipError_t launch_mlp_precond(const Dev&, const LearnDev&, hipStream_t) { return hipSuccess; }
hipError_t launch_mlp_grad(const LearnDev&, const SampleSrc&, int, float*, double*, float*, hipStream_t) {
  return hipSuccess;
}
hipError_t launch_adam(const LearnDev&, const float*, float, int, hipStream_t) { return hipSuccess; }
hipError_t launch_to_bf16(const LearnDev&, hipStream_t) { return hipSuccess; }
int mlp_tiles(int n) { return (n + 255) / 256; }
#endif
}  // namespace sqrtba

namespace {

struct Rng {
  uint64_t s;
  uint64_t next() {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    return s;
  }
  int64_t below(int64_t n) { return (int64_t)(next() % (uint64_t)n); }
};

int check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    std::exit(1);
  }
  return 0;
}

// `parts` problems of `cams_per` cameras and `pts_per` landmarks, k in [kmin, kmax].
void run_case(uint64_t seed, int parts, int cams_per, int pts_per, int kmin, int kmax, int test_kernel) {
  Rng rng{seed * 2654435761ull + 7};
  sqrtba_options opt;
  SQRTBA_API(default_options)(&opt);
  opt.max_lm_iters = 6;
  opt.pcg_max_iters = 20;
  opt.pcg_check_every = 8;
  opt.pcg_test_kernel = test_kernel;
  sqrtba_ctx* c = nullptr;
  check(SQRTBA_API(create)(&c, &opt, nullptr) == SQRTBA_OK && c, "create");
  std::vector<int64_t> co{0}, po{0};
  for (int p = 0; p < parts; ++p) {
    co.push_back(co.back() + cams_per);
    po.push_back(po.back() + pts_per);
  }
  if (parts > 1) check(SQRTBA_API(set_problems)(c, parts, co.data(), po.data()) == SQRTBA_OK, "set_problems");
  const int64_t NC = co.back(), NL = po.back();
  std::vector<real> cams(9 * NC), pts(3 * NL);
  for (auto& v : cams) v = (real)((rng.below(2000) - 1000) * 1e-3);
  for (auto& v : pts) v = (real)((rng.below(2000) - 1000) * 1e-3);
  check(SQRTBA_API(set_cameras)(c, NC, cams.data()) == SQRTBA_OK, "set_cameras");
  check(SQRTBA_API(set_landmarks)(c, NL, pts.data()) == SQRTBA_OK, "set_landmarks");
  std::vector<int32_t> oc, op;
  std::vector<real> uv;
  for (int p = 0; p < parts; ++p)
    for (int64_t l = po[p]; l < po[p + 1]; ++l) {
      const int k = (int)std::min<int64_t>(cams_per, kmin + rng.below(kmax - kmin + 1));
      std::vector<int> perm(cams_per);
      for (int i = 0; i < cams_per; ++i) perm[i] = i;
      for (int i = 0; i < k; ++i) std::swap(perm[i], perm[i + rng.below(cams_per - i)]);
      for (int i = 0; i < k; ++i) {
        oc.push_back((int32_t)(co[p] + perm[i]));
        op.push_back((int32_t)l);
        uv.push_back((real)rng.below(100));
        uv.push_back((real)rng.below(100));
      }
    }
  check(SQRTBA_API(set_observations)(c, (int64_t)oc.size(), oc.data(), op.data(), uv.data()) == SQRTBA_OK,
        "set_observations");
  // the autotuner: every launch shape, graph capture of back-to-back products
  sqrtba_tuning best;
  std::vector<sqrtba_tuning_trial> trials(4);  // fewer slots than trials: the copy is bounded
  int32_t n_trials = 0;
  check(SQRTBA_API(autotune)(c, 3, &best, trials.data(), (int32_t)trials.size(), &n_trials) == SQRTBA_OK,
        "autotune");
  check(n_trials >= 1, "autotune trials");
  // the stages one by one
  std::vector<double> cost(parts), lam(parts, 1e-4), pred(parts), newc(parts), rel(parts);
  std::vector<int32_t> its(parts), st(parts);
  std::vector<uint8_t> acc(parts, 1);
  check(SQRTBA_API(linearize)(c, cost.data()) == SQRTBA_OK, "linearize");
  check(SQRTBA_API(marginalize)(c) == SQRTBA_OK, "marginalize");
  check(SQRTBA_API(damp)(c, lam.data()) == SQRTBA_OK, "damp");
  check(SQRTBA_API(solve)(c, its.data(), rel.data(), st.data()) == SQRTBA_OK, "solve");
  check(SQRTBA_API(back_substitute)(c, pred.data()) == SQRTBA_OK, "back_substitute");
  check(SQRTBA_API(update)(c, newc.data()) == SQRTBA_OK, "update");
  check(SQRTBA_API(commit)(c, acc.data()) == SQRTBA_OK, "commit");
  // the whole LM loop, twice (the second on a context whose pinned slices and graph exist)
  std::vector<sqrtba_lm_report> rep(parts);
  for (int r = 0; r < 2; ++r) check(SQRTBA_API(lm_solve)(c, rep.data()) == SQRTBA_OK, "lm_solve");
  std::vector<double> tol(parts, 1.0);
  check(SQRTBA_API(lm_solve_tracked)(c, tol.data(), rep.data()) == SQRTBA_OK, "lm_solve_tracked");
  int32_t nh = 0;
  check(SQRTBA_API(get_lm_history)(c, 0, nullptr, 0, &nh) == SQRTBA_OK, "history size");
  std::vector<sqrtba_lm_record> hist((size_t)std::max(1, nh));
  check(SQRTBA_API(get_lm_history)(c, 0, hist.data(), nh, &nh) == SQRTBA_OK, "history");
  // the learned preconditioner: traces of the solves, training, learned solves with fallbacks
  check(SQRTBA_API(mlp_init)(c, 3) == SQRTBA_OK, "mlp_init");
  check(SQRTBA_API(pcg_trace)(c, 2, 8) == SQRTBA_OK, "pcg_trace");
  check(SQRTBA_API(lm_solve)(c, rep.data()) == SQRTBA_OK, "lm_solve (traced)");
  int32_t ns = 0, nr = 0;
  check(SQRTBA_API(trace_size)(c, &ns, &nr) == SQRTBA_OK, "trace_size");
  std::vector<double> losses(3);
  if (nr > 0) check(SQRTBA_API(mlp_train)(c, 3, 64, 1e-3, 5, losses.data()) == SQRTBA_OK, "mlp_train");
  std::vector<float> theta(SQRTBA_API(mlp_num_params)());
  check(SQRTBA_API(mlp_get_params)(c, theta.data()) == SQRTBA_OK, "mlp_get_params");
  check(SQRTBA_API(mlp_set_params)(c, theta.data()) == SQRTBA_OK, "mlp_set_params");
  check(SQRTBA_API(set_preconditioner)(c, 1) == SQRTBA_OK, "set_preconditioner");
  check(SQRTBA_API(lm_solve)(c, rep.data()) == SQRTBA_OK, "lm_solve (learned)");
  int64_t ls = 0, fb = 0, wi = 0;
  check(SQRTBA_API(learned_stats)(c, &ls, &fb, &wi) == SQRTBA_OK, "learned_stats");
  check(SQRTBA_API(set_preconditioner)(c, 0) == SQRTBA_OK, "set_preconditioner back");
  // inspection exports and the product without allocation
  {
    const int64_t nc9 = 9 * NC;
    std::vector<float> v(2 * nc9, 0.5f), out(2 * nc9), rhs(nc9), minv(81 * NC);
    check(SQRTBA_API(linearize)(c, cost.data()) == SQRTBA_OK, "linearize (exports)");
    check(SQRTBA_API(marginalize)(c) == SQRTBA_OK, "marginalize (exports)");
    check(SQRTBA_API(damp)(c, lam.data()) == SQRTBA_OK, "damp (exports)");
    check(SQRTBA_API(debug_rcs_matvec)(c, 2, v.data(), out.data()) == SQRTBA_OK, "debug_rcs_matvec");
    check(SQRTBA_API(rcs_matvec_noalloc)(c, v.data(), out.data()) == SQRTBA_OK, "rcs_matvec_noalloc");
    check(SQRTBA_API(solve)(c, its.data(), rel.data(), st.data()) == SQRTBA_OK, "solve (exports)");
    check(SQRTBA_API(debug_rhs)(c, rhs.data()) == SQRTBA_OK, "debug_rhs");
    check(SQRTBA_API(debug_precond)(c, minv.data()) == SQRTBA_OK, "debug_precond");
  }
  // a subset of the problems active
  if (parts > 1) {
    std::vector<uint8_t> mask(parts, 0);
    mask[1] = 1;
    check(SQRTBA_API(set_active)(c, mask.data()) == SQRTBA_OK, "set_active");
    check(SQRTBA_API(lm_solve)(c, rep.data()) == SQRTBA_OK, "lm_solve (subset)");
  }
  SQRTBA_API(destroy)(c);
}

}  // namespace

int main() {
  int n = 0;
  for (int t = -1; t <= 1; ++t) {
    run_case(1 + t, 1, 8, 200, 2, 8, t);          // one small problem
    run_case(11 + t, 5, 12, 60, 2, 12, t);        // a batch of uneven problems
    run_case(21 + t, 1, 300, 40, 100, 300, t);    // class-5 landmarks: row blocks, chunked QR
    n += 3;
  }
  std::printf("host LM loop sanitizer driver: %d cases ok\n", n);
  return 0;
}
