// Host-side bookkeeping and workspace layout of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (CPU only, no GPU call): the library's host code is
// compiled into this program, and a context is driven through problem definition,
// bookkeeping (sort by landmark and camera, CSR, size classes, row-block and chunk
// job lists), the explicit Schur complement's camera-pair structure and the
// workspace layout of every landmark-block form, on random and degenerate inputs.
#include "../../paper_2103_01843_amd/csrc/api.cpp"

#include <cstdlib>

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

// One problem (or a batch of `parts` problems) with k in [kmin, kmax] per landmark.
void run_case(uint64_t seed, int parts, int cams_per, int pts_per, int kmin, int kmax, int mode) {
  Rng rng{seed * 2654435761ull + 1};
  sqrtba_ctx c;
  SQRTBA_API(default_options)(&c.opt);
  c.opt.landmark_blocks = mode;
  std::vector<int64_t> co{0}, po{0};
  for (int p = 0; p < parts; ++p) {
    co.push_back(co.back() + cams_per);
    po.push_back(po.back() + pts_per);
  }
  if (parts > 1) check(SQRTBA_API(set_problems)(&c, parts, co.data(), po.data()) == SQRTBA_OK, "set_problems");
  const int64_t NC = co.back(), NL = po.back();
  std::vector<real> cams(9 * NC), pts(3 * NL);
  for (auto& v : cams) v = (real)((rng.below(2000) - 1000) * 1e-3);
  for (auto& v : pts) v = (real)((rng.below(2000) - 1000) * 1e-3);
  check(SQRTBA_API(set_cameras)(&c, NC, cams.data()) == SQRTBA_OK, "set_cameras");
  check(SQRTBA_API(set_landmarks)(&c, NL, pts.data()) == SQRTBA_OK, "set_landmarks");
  std::vector<int32_t> oc, op;
  std::vector<real> uv;
  for (int p = 0; p < parts; ++p)
    for (int64_t l = po[p]; l < po[p + 1]; ++l) {
      const int k = std::min<int64_t>(cams_per, kmin + rng.below(kmax - kmin + 1));
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
  // shuffle the observations
  for (size_t i = oc.size(); i > 1; --i) {
    const size_t j = (size_t)rng.below((int64_t)i);
    std::swap(oc[i - 1], oc[j]);
    std::swap(op[i - 1], op[j]);
    std::swap(uv[2 * (i - 1)], uv[2 * j]);
    std::swap(uv[2 * (i - 1) + 1], uv[2 * j + 1]);
  }
  const int st = SQRTBA_API(set_observations)(&c, (int64_t)oc.size(), oc.data(), op.data(), uv.data());
  if (kmax > SQRTBA_MAX_OBS_PER_LANDMARK) {
    check(st == SQRTBA_E_UNSUPPORTED, "oversized landmark rejected");
    return;
  }
  check(st == SQRTBA_OK, "set_observations");
  if (mode == 2) check(build_sc(&c) == SQRTBA_OK, "build_sc");
  uint64_t bytes = 0;
  check(SQRTBA_API(workspace_bytes)(&c, &bytes) == SQRTBA_OK && bytes > 0, "workspace_bytes");
  // CSR and slot invariants
  const HostData& h = c.h;
  check((int64_t)h.lm_off.size() == NL + 1 && h.lm_off.back() == h.NO, "landmark CSR");
  int64_t sum_k = 0;
  for (int64_t s = 0; s < h.NS; ++s) {
    sum_k += h.slot_k[s];
    if (s) check(h.slot_k[s] <= h.slot_k[s - 1], "slots by decreasing k");
  }
  check(sum_k == h.NO, "every active observation in one slot");
  // invalid inputs leave the state unchanged and are reported
  if (!oc.empty()) {
    std::vector<int32_t> bad = oc;
    bad[0] = (int32_t)NC;
    check(SQRTBA_API(set_observations)(&c, (int64_t)bad.size(), bad.data(), op.data(), uv.data()) == SQRTBA_E_INVALID,
          "camera index out of range");
    check(c.h.NO == h.NO, "state unchanged after an error");
  }
}

}  // namespace

int main() {
  int n = 0;
  for (int mode = 0; mode < 3; ++mode) {
    run_case(1 + mode, 1, 8, 200, 2, 8, mode);                 // small ring-like problem
    run_case(11 + mode, 5, 12, 60, 2, 12, mode);               // a batch of uneven problems
    run_case(21 + mode, 1, 300, 40, 100, 300, mode == 2 ? 0 : mode);  // class-5 landmarks: chunks and row blocks
    run_case(31 + mode, 1, 4, 50, 1, 4, mode);                 // inactive landmarks (k = 1) and unused cameras
    n += 4;
  }
  run_case(41, 1, 600, 3, 513, 520, 0);                       // more observations than supported
  std::printf("host bookkeeping sanitizer driver: %d cases ok\n", n + 1);
  return 0;
}
