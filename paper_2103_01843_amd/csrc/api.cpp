// Host side of libsqrtba.so (and, built with SQRTBA_FP64, of libsqrtba64.so):
// the C ABI of include/sqrtba.h (include/sqrtba64.h), observation
// bookkeeping, device memory layout and the Levenberg-Marquardt loop.
// Every floating-point step of the solve runs in the HIP kernels of
// kernels.hip; the host only sorts indices, moves data, reads back per-problem
// scalars and takes the accept/reject decisions of Sec. 6.1.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#ifdef SQRTBA_FP64
// libsqrtba64.so: the same host code over FP64 kernels, with its own context type
#define sqrtba_ctx sqrtba64_ctx
#include "../../include/sqrtba64.h"
#define SQRTBA_API(name) sqrtba64_##name
#else
#include "../../include/sqrtba.h"
#define SQRTBA_API(name) sqrtba_##name
#endif
#include "device.h"
#include "learned.h"

using namespace sqrtba;

static_assert(NOALLOC_SCRATCH_BYTES == SQRTBA_NOALLOC_SCRATCH_BYTES, "no-allocation scratch size of the header");

namespace {

constexpr int32_t kVersion = 1;

struct HostData {
  // problem partition
  int32_t P = 1;
  std::vector<int64_t> cam_off{0, 0}, pt_off{0, 0};
  bool problems_set = false;
  // inputs
  int64_t NC = -1, NL = -1;
  std::vector<real> cams_bal;  // NC * 9
  std::vector<real> pts;       // NL * 3
  // bookkeeping
  bool obs_set = false;
  int64_t n_obs_in = 0, NO = 0, NS = 0;
  std::vector<int64_t> obs_perm, lm_off;
  std::vector<uint8_t> lm_active, cam_active;
  std::vector<int32_t> ocam, olm;
  std::vector<real> ouv;
  std::vector<int32_t> cam_obs_off, cam_obs_idx, cam_prob, lm_prob, prob_cam_off, prob_lm_off;
  std::vector<int32_t> slot_lm, slot_k, slot_obs0, slot_prob, lm_slot;
  std::vector<int64_t> slot_boff, slot_toff;
  std::vector<int32_t> slot_zoff, cam_zpos;
  std::vector<float> cam_stats;  // NC * 4 features of the camera's observation graph
  WorkClass wc[NUM_CLASSES];
  std::vector<int32_t> hjob;   // (slot, row block) pairs of the row-block product (capacity)
  std::vector<int32_t> qjob;   // (slot, first row | end row << 16) chunks of the class-5 QR
  std::vector<int64_t> hz_off; // per slot with k >= ROWS_MIN_K, offset of its partial outputs
  int64_t hz_floats = 0;
  int64_t z_floats = 0;        // elements of the product's per-observation output area (explicit blocks)
  int64_t poolB = 0, poolT = 0;
  // explicit Schur complement (landmark_blocks = 2): camera-pair blocks of the
  // reduced matrix, built on demand (O(sum k^2) host work and memory)
  struct Sc {
    bool built = false;
    int64_t noff = 0;
    std::vector<int32_t> coff;     // noff + 1
    std::vector<int32_t> contrib;  // 4 per contribution: record a, record b, slot, 0
    std::vector<int32_t> rowoff;   // NC + 1
    std::vector<int32_t> rowent;   // 2 per entry: block | transposed << 31, other camera
    std::vector<int32_t> blk_prob; // problem of each off-diagonal block
  } sc;
};

struct Arena {
  void* base = nullptr;
  uint64_t bytes = 0;
  bool owned = false;
};

}  // namespace

// slices of 8 bytes per problem in the pinned staging buffer (pinned_slice)
constexpr int PINNED_SLICES = 10;

struct sqrtba_ctx {
  sqrtba_options opt;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t side = nullptr;  // side stream for the largest landmark blocks
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int device = 0;
  void* noalloc_scratch = nullptr;  // device address of the no-allocation product's scratch on `device`
  std::string err;
  HostData h;
  Arena arena;
  bool uploaded = false;
  Dev d{};
  Launch L{};
  // pinned host staging for per-problem scalars
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  // coherent pinned host memory the PCG update kernel writes the done flags to
  int32_t* done_host = nullptr;
  int32_t* done_host_dev = nullptr;
  int64_t done_host_n = 0;
  // pipeline state
  bool linearized = false, marginalized = false, damped = false, solved = false, backsubbed = false,
       updated = false;
  bool solve_pending = false;  // a solve's outcome is on its way to the pinned slices 5, 8 and 9
  std::vector<uint8_t> active;
  // PCG graph
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  bool graph_profiled = false;
  // stage profiler
  bool prof_on = false;
  sqrtba_profile prof{};
  struct Pending {
    int stage;
    hipEvent_t a, b;
    double bytes;
    int64_t units;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  // per-problem algorithmic bytes of one matvec and one marginalization
  std::vector<double> mv_bytes, qr_bytes;
  std::vector<int64_t> blocks;
  bool snapshot = false;
  // LM history
  std::vector<std::vector<sqrtba_lm_record>> history;
  // learned preconditioner
  struct Learned {
    bool alloc = false;
    float* w32 = nullptr;
    uint16_t* wbf = nullptr;
    float *adam_m = nullptr, *adam_v = nullptr, *grad = nullptr;
    float* part = nullptr;
    double* loss_part = nullptr;
    int part_tiles = 0;
    int adam_step = 0;
    int mode = 0;  // 0 block-Jacobi, 1 learned with block-Jacobi fallback
    // trace store
    int max_solves = 0, iters_per_solve = 0, n_solves = 0, n_records = 0, cur_solve = -1, cur_iter = 0;
    float *t_feat = nullptr, *t_lfac = nullptr, *t_p = nullptr, *t_q = nullptr;
    int32_t* rec_solve = nullptr;
    std::vector<int32_t> h_rec_solve;
    int32_t *s_rec = nullptr, *s_cam = nullptr;
    int s_cap = 0;
    std::vector<int32_t> last_plain_iters;
    std::vector<int32_t> last_plain_status;
    int64_t learned_solves = 0, fallbacks = 0, wasted_iters = 0;
  } ln;
};

namespace {

int fail(sqrtba_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(ctx, SQRTBA_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)              \
  do {                         \
    int s_ = (expr);           \
    if (s_ != SQRTBA_OK) return s_; \
  } while (0)

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Rodrigues' formula in double (half-angle form; series below 1e-8).
void so3_exp_d(const double w[3], double R[9]) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = std::sqrt(th2);
  double a, b;
  if (th < 1e-8) {
    a = 1.0;
    b = 0.5;
  } else {
    const double sh = std::sin(0.5 * th);
    a = std::sin(th) / th;
    b = 2.0 * sh * sh / th2;
  }
  const double W[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int q = 0; q < 3; ++q) s += W[3 * i + q] * W[3 * q + j];
      R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * W[3 * i + j] + b * s;
    }
}

// Angle-axis of a rotation matrix, valid up to and at angle pi.  The angle is
// atan2(|v| / 2, (tr R - 1) / 2) with v the antisymmetric part (acos of the
// trace alone loses half the digits near pi); for angles above pi/2 the axis
// comes from the symmetric part, cos(t) I + (1 - cos(t)) a a^T, with the sign
// of v.
void so3_log_d(const double M[9], double w[3]) {
  const double c = 0.5 * (M[0] + M[4] + M[8] - 1.0);
  const double v[3] = {M[7] - M[5], M[2] - M[6], M[3] - M[1]};
  const double s = 0.5 * std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double th = std::atan2(s, c);
  if (th < 1e-8) {
    for (int i = 0; i < 3; ++i) w[i] = 0.5 * v[i];
  } else if (c >= 0.0) {
    for (int i = 0; i < 3; ++i) w[i] = th * v[i] / (2.0 * s);
  } else {
    double B[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        B[3 * i + j] = (0.5 * (M[3 * i + j] + M[3 * j + i]) - (i == j ? c : 0.0)) / (1.0 - c);
    int i = 0;
    if (B[4] > B[3 * i + i]) i = 1;
    if (B[8] > B[3 * i + i]) i = 2;
    double a[3];
    const double nrm = std::sqrt(std::max(B[3 * i + i], 1e-300));
    for (int j = 0; j < 3; ++j) a[j] = B[3 * j + i] / nrm;
    const double an = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double dot = 0;
    for (int j = 0; j < 3; ++j) {
      a[j] /= an;
      dot += a[j] * v[j];
    }
    const double sg = dot < 0 ? -1.0 : 1.0;
    for (int j = 0; j < 3; ++j) w[j] = sg * th * a[j];
  }
}

int64_t width_of_h(int64_t k) { return (9 * k + 3) & ~int64_t(3); }

// (slot, row block) jobs of the row-block product for the first nrows slots
// (the landmarks with the most observations) and blocks of `rows` rows.
void build_hjobs(const HostData& h, int rows, int64_t nrows, std::vector<int32_t>& jobs) {
  jobs.clear();
  for (int64_t sl = 0; sl < nrows; ++sl) {
    const int64_t k = h.slot_k[sl];
    const int64_t nblk = (2 * k + rows - 1) / rows;
    for (int64_t r = 0; r < nblk; ++r) {
      jobs.push_back((int32_t)sl);
      jobs.push_back((int32_t)r);
    }
  }
}

// Number of leading slots with k >= kmin (slots are ordered by decreasing k).
int64_t slots_with_k_at_least(const HostData& h, int64_t kmin) {
  int64_t n = 0;
  while (n < h.NS && h.slot_k[n] >= kmin) ++n;
  return n;
}

// ------------------------------------------------------------ bookkeeping

int build_sc(sqrtba_ctx* c);

int build_bookkeeping(sqrtba_ctx* c, int64_t n, const int32_t* cam, const int32_t* pt, const real* uv) {
  HostData& h = c->h;
  if (n <= 0) return fail(c, SQRTBA_E_INVALID, "n_obs must be positive");
  if (!cam || !pt || !uv) return fail(c, SQRTBA_E_INVALID, "null observation array");
  std::vector<int32_t> cprob(h.NC), pprob(h.NL);
  for (int32_t p = 0; p < h.P; ++p) {
    for (int64_t i = h.cam_off[p]; i < h.cam_off[p + 1]; ++i) cprob[i] = p;
    for (int64_t i = h.pt_off[p]; i < h.pt_off[p + 1]; ++i) pprob[i] = p;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (cam[i] < 0 || cam[i] >= h.NC) return fail(c, SQRTBA_E_INVALID, "observation %lld: camera %d out of range", (long long)i, cam[i]);
    if (pt[i] < 0 || pt[i] >= h.NL) return fail(c, SQRTBA_E_INVALID, "observation %lld: landmark %d out of range", (long long)i, pt[i]);
    if (!std::isfinite(uv[2 * i]) || !std::isfinite(uv[2 * i + 1]))
      return fail(c, SQRTBA_E_NONFINITE, "observation %lld: non-finite pixel", (long long)i);
    if (cprob[cam[i]] != pprob[pt[i]])
      return fail(c, SQRTBA_E_INVALID, "observation %lld links problems %d and %d", (long long)i, cprob[cam[i]], pprob[pt[i]]);
  }
  // sort by (landmark, camera)
  std::vector<int64_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = i;
  std::vector<uint64_t> key(n);
  for (int64_t i = 0; i < n; ++i) key[i] = ((uint64_t)(uint32_t)pt[i] << 32) | (uint32_t)cam[i];
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return key[a] < key[b] || (key[a] == key[b] && a < b); });
  for (int64_t i = 1; i < n; ++i)
    if (key[order[i]] == key[order[i - 1]])
      return fail(c, SQRTBA_E_INVALID, "duplicate observation of landmark %d by camera %d", pt[order[i]], cam[order[i]]);
  std::vector<int64_t> count(h.NL, 0);
  for (int64_t i = 0; i < n; ++i) count[pt[i]]++;
  for (int64_t l = 0; l < h.NL; ++l)
    if (count[l] > SQRTBA_MAX_OBS_PER_LANDMARK)
      return fail(c, SQRTBA_E_UNSUPPORTED, "landmark %lld has %lld observations (max %d)", (long long)l,
                  (long long)count[l], SQRTBA_MAX_OBS_PER_LANDMARK);

  HostData nb = h;  // build into a copy so errors leave the state unchanged
  nb.n_obs_in = n;
  nb.lm_active.assign(h.NL, 0);
  nb.lm_off.assign(h.NL + 1, 0);
  for (int64_t l = 0; l < h.NL; ++l) {
    nb.lm_active[l] = count[l] >= 2;
    nb.lm_off[l + 1] = nb.lm_off[l] + (nb.lm_active[l] ? count[l] : 0);
  }
  nb.obs_perm.clear();
  for (int64_t i = 0; i < n; ++i)
    if (nb.lm_active[pt[order[i]]]) nb.obs_perm.push_back(order[i]);
  nb.NO = (int64_t)nb.obs_perm.size();
  if (nb.NO > INT32_MAX / 64) return fail(c, SQRTBA_E_UNSUPPORTED, "too many observations");
  nb.ocam.resize(nb.NO);
  nb.olm.resize(nb.NO);
  nb.ouv.resize(2 * nb.NO);
  for (int64_t j = 0; j < nb.NO; ++j) {
    const int64_t i = nb.obs_perm[j];
    nb.ocam[j] = cam[i];
    nb.olm[j] = pt[i];
    nb.ouv[2 * j] = uv[2 * i];
    nb.ouv[2 * j + 1] = uv[2 * i + 1];
  }
  // per-camera lists of sorted positions (counting sort keeps them ascending)
  nb.cam_obs_off.assign(h.NC + 1, 0);
  for (int64_t j = 0; j < nb.NO; ++j) nb.cam_obs_off[nb.ocam[j] + 1]++;
  for (int64_t q = 0; q < h.NC; ++q) nb.cam_obs_off[q + 1] += nb.cam_obs_off[q];
  nb.cam_obs_idx.assign(nb.NO, 0);
  {
    std::vector<int32_t> fill(nb.cam_obs_off.begin(), nb.cam_obs_off.end() - 1);
    for (int64_t j = 0; j < nb.NO; ++j) nb.cam_obs_idx[fill[nb.ocam[j]]++] = (int32_t)j;
  }
  nb.cam_active.assign(h.NC, 0);
  for (int64_t q = 0; q < h.NC; ++q) nb.cam_active[q] = nb.cam_obs_off[q + 1] > nb.cam_obs_off[q];
  nb.cam_prob = cprob;
  nb.lm_prob = pprob;
  nb.prob_cam_off.resize(h.P + 1);
  nb.prob_lm_off.resize(h.P + 1);
  for (int32_t p = 0; p <= h.P; ++p) {
    nb.prob_cam_off[p] = (int32_t)h.cam_off[p];
    nb.prob_lm_off[p] = (int32_t)h.pt_off[p];
  }
  // slots: active landmarks by decreasing k (ties by landmark index)
  std::vector<int32_t> act;
  for (int64_t l = 0; l < h.NL; ++l)
    if (nb.lm_active[l]) act.push_back((int32_t)l);
  std::stable_sort(act.begin(), act.end(), [&](int32_t a, int32_t b) { return count[a] > count[b]; });
  nb.NS = (int64_t)act.size();
  nb.slot_lm = act;
  nb.slot_k.resize(nb.NS);
  nb.slot_obs0.resize(nb.NS);
  nb.slot_prob.resize(nb.NS);
  nb.slot_boff.resize(nb.NS);
  nb.slot_toff.resize(nb.NS);
  nb.lm_slot.assign(h.NL, -1);
  nb.slot_zoff.resize(nb.NS);
  int64_t ob = 0, ot = 0, oz = 0;
  for (int64_t s = 0; s < nb.NS; ++s) {
    const int32_t l = act[s];
    const int64_t k = count[l];
    nb.slot_k[s] = (int32_t)k;
    nb.slot_obs0[s] = (int32_t)nb.lm_off[l];
    nb.slot_prob[s] = pprob[l];
    nb.slot_boff[s] = ob;
    nb.slot_toff[s] = ot;
    nb.lm_slot[l] = (int32_t)s;
    const int64_t W = width_of_h(k);
    nb.slot_zoff[s] = (int32_t)oz;
    // each landmark's rows start on a 128-byte line, so neighbouring blocks
    // never share a cache line (the QR writes them from different wavefronts)
    ob += (2 * k * W + 31) & ~int64_t(31);
    ot += (3 * W + 31) & ~int64_t(31);
    oz += W;
  }
  if (oz > 54 * nb.NO || oz > INT32_MAX) return fail(c, SQRTBA_E_UNSUPPORTED, "product output area too large");
  nb.z_floats = oz;
  // offsets of each camera's observation outputs, in camera order
  {
    std::vector<int32_t> zpos_of_obs(nb.NO);
    for (int64_t sl = 0; sl < nb.NS; ++sl)
      for (int64_t o = 0; o < nb.slot_k[sl]; ++o)
        zpos_of_obs[nb.slot_obs0[sl] + o] = nb.slot_zoff[sl] + (int32_t)(9 * o);
    nb.cam_zpos.resize(nb.NO);
    for (int64_t q = 0; q < nb.NO; ++q) nb.cam_zpos[q] = zpos_of_obs[nb.cam_obs_idx[q]];
    // each camera's outputs are summed in increasing address order (its reads
    // then move through memory in one direction)
    for (int64_t cc = 0; cc < h.NC; ++cc)
      std::sort(nb.cam_zpos.begin() + nb.cam_obs_off[cc], nb.cam_zpos.begin() + nb.cam_obs_off[cc + 1]);
  }
  nb.poolB = ob;
  nb.poolT = ot;
  // size classes: contiguous k ranges, and slots are sorted by decreasing k
  for (int cl = NUM_CLASSES - 1; cl >= 0; --cl) {
    int64_t s = 0;
    while (s < nb.NS && class_of_k(nb.slot_k[s]) != cl) ++s;
    nb.wc[cl].first_slot = (int)s;
    while (s < nb.NS && class_of_k(nb.slot_k[s]) == cl) ++s;
    nb.wc[cl].slots = (int)(s - nb.wc[cl].first_slot);
  }
  // row-block product: partial outputs per row block for every landmark that
  // can take it (k >= ROWS_MIN_K, a prefix of the slots), sized for the
  // smallest block (HUGE_ROWS_MIN rows); the job list is built per shape
  nb.hz_off.clear();
  nb.hz_floats = 0;
  const int64_t n45 = slots_with_k_at_least(nb, ROWS_MIN_K);
  for (int64_t sl = 0; sl < n45; ++sl) {
    const int64_t k = nb.slot_k[sl];
    nb.hz_off.push_back(nb.hz_floats);
    nb.hz_floats += ((2 * k + HUGE_ROWS_MIN - 1) / HUGE_ROWS_MIN) * width_of_h(k);
  }
  build_hjobs(nb, HUGE_ROWS_MIN, n45, nb.hjob);
  if (nb.hjob.size() / 2 > (size_t)INT32_MAX / 2) return fail(c, SQRTBA_E_UNSUPPORTED, "too many row blocks");
  // QR of class 5 (explicit blocks) in row chunks of about QR_CHUNK_BYTES each,
  // so that no single workgroup writes a whole multi-megabyte block
  nb.qjob.clear();
  for (int64_t sl = nb.wc[5].first_slot; sl < nb.wc[5].first_slot + nb.wc[5].slots; ++sl) {
    const int64_t nrows = 2 * nb.slot_k[sl];
    const int64_t rows = std::max<int64_t>(1, QR_CHUNK_BYTES / ((int64_t)sizeof(real) * width_of_h(nb.slot_k[sl])));
    for (int64_t r = 0; r < nrows; r += rows) {
      nb.qjob.push_back((int32_t)sl);
      nb.qjob.push_back((int32_t)(r | (std::min(nrows, r + rows) << 16)));
    }
  }
  if (nb.qjob.size() / 2 > (size_t)INT32_MAX) return fail(c, SQRTBA_E_UNSUPPORTED, "too many QR chunks");
  // camera statistics for the learned preconditioner: observations, covisible
  // cameras (bitsets per problem), mean and max log k over the camera's landmarks
  nb.cam_stats.assign(4 * h.NC, 0.f);
  for (int32_t p = 0; p < h.P; ++p) {
    const int64_t c0 = h.cam_off[p], nc = h.cam_off[p + 1] - c0, words = (nc + 63) / 64;
    if (nc == 0) continue;
    std::vector<uint64_t> bits(nc * words, 0), lm(words, 0);
    for (int64_t l = h.pt_off[p]; l < h.pt_off[p + 1]; ++l) {
      if (!nb.lm_active[l]) continue;
      const int64_t b = nb.lm_off[l], e = nb.lm_off[l + 1];
      int64_t wlo = words, whi = -1;
      for (int64_t o = b; o < e; ++o) {
        const int64_t cc = nb.ocam[o] - c0;
        lm[cc >> 6] |= uint64_t(1) << (cc & 63);
        wlo = std::min(wlo, cc >> 6);
        whi = std::max(whi, cc >> 6);
      }
      for (int64_t o = b; o < e; ++o) {
        uint64_t* row = bits.data() + (nb.ocam[o] - c0) * words;
        for (int64_t w = wlo; w <= whi; ++w) row[w] |= lm[w];
      }
      for (int64_t w = wlo; w <= whi; ++w) lm[w] = 0;
    }
    for (int64_t cc = 0; cc < nc; ++cc) {
      const int64_t ci = c0 + cc;
      int64_t cov = 0;
      for (int64_t w = 0; w < words; ++w) cov += __builtin_popcountll(bits[cc * words + w]);
      const int64_t nob = nb.cam_obs_off[ci + 1] - nb.cam_obs_off[ci];
      double sk = 0, mk = 0;
      for (int64_t i = nb.cam_obs_off[ci]; i < nb.cam_obs_off[ci + 1]; ++i) {
        const int32_t l = nb.olm[nb.cam_obs_idx[i]];
        const double lk = std::log((double)count[l]);
        sk += lk;
        mk = std::max(mk, lk);
      }
      nb.cam_stats[4 * ci + 0] = (float)std::log1p((double)nob);
      nb.cam_stats[4 * ci + 1] = (float)std::log1p((double)std::max<int64_t>(cov - 1, 0));
      nb.cam_stats[4 * ci + 2] = nob ? (float)(sk / nob) : 0.f;
      nb.cam_stats[4 * ci + 3] = (float)mk;
    }
  }
  nb.obs_set = true;
  nb.sc = HostData::Sc{};
  h = std::move(nb);
  if (c->opt.landmark_blocks == 2) TRY(build_sc(c));
  return SQRTBA_OK;
}

// ------------------------------------------------------------ device memory

struct Layout {
  uint64_t total = 0;
  uint64_t take(uint64_t bytes) {
    const uint64_t at = total;
    total += (bytes + 255) & ~uint64_t(255);
    return at;
  }
};

template <typename T>
T* at(void* base, uint64_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// Offsets of every device array; when base is null only the size is computed.
// Camera-pair blocks of the explicit Schur complement: every pair a < b of a
// landmark's observations (cameras ascending) contributes G_a H~^-1 G_b^T to
// block (camera a, camera b).  Contributions are sorted by (camera a, camera b)
// with a stable two-pass counting sort, so each block sums them in slot order;
// each camera's row lists its diagonal block, then its blocks in block order.
int build_sc(sqrtba_ctx* c) {
  HostData& h = c->h;
  if (h.sc.built) return SQRTBA_OK;
  int64_t n = 0;
  for (int64_t s = 0; s < h.NS; ++s) n += (int64_t)h.slot_k[s] * (h.slot_k[s] - 1) / 2;
  if (n > (int64_t)1 << 30)
    return fail(c, SQRTBA_E_UNSUPPORTED, "explicit Schur complement with %lld pair contributions", (long long)n);
  std::vector<int32_t> ca(n), cb(n), ra(n), rb(n), sl(n);
  {
    int64_t e = 0, r0 = 0;
    for (int64_t s = 0; s < h.NS; ++s) {
      const int64_t k = h.slot_k[s], o0 = h.slot_obs0[s];
      for (int64_t a = 0; a < k; ++a)
        for (int64_t b = a + 1; b < k; ++b) {
          ca[e] = h.ocam[o0 + a];
          cb[e] = h.ocam[o0 + b];
          ra[e] = (int32_t)(r0 + a);
          rb[e] = (int32_t)(r0 + b);
          sl[e] = (int32_t)s;
          ++e;
        }
      r0 += k;
    }
  }
  const int64_t NC = h.NC;
  std::vector<int64_t> order(n), tmp(n), cnt(NC + 1);
  for (int64_t e = 0; e < n; ++e) tmp[e] = e;
  for (int pass = 0; pass < 2; ++pass) {  // by camera b, then (stable) by camera a
    const std::vector<int32_t>& key = pass == 0 ? cb : ca;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t e = 0; e < n; ++e) cnt[key[tmp[e]] + 1]++;
    for (int64_t q = 0; q < NC; ++q) cnt[q + 1] += cnt[q];
    for (int64_t e = 0; e < n; ++e) order[cnt[key[tmp[e]]]++] = tmp[e];
    tmp.swap(order);
  }
  HostData::Sc sc;
  sc.contrib.resize(4 * n);
  std::vector<int32_t> bca, bcb;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t e = tmp[i];
    if (i == 0 || ca[e] != bca.back() || cb[e] != bcb.back()) {
      sc.coff.push_back((int32_t)i);
      bca.push_back(ca[e]);
      bcb.push_back(cb[e]);
    }
    sc.contrib[4 * i + 0] = ra[e];
    sc.contrib[4 * i + 1] = rb[e];
    sc.contrib[4 * i + 2] = sl[e];
    sc.contrib[4 * i + 3] = 0;
  }
  sc.noff = (int64_t)bca.size();
  sc.coff.push_back((int32_t)n);
  if (sc.noff + NC > (int64_t)INT32_MAX / 81)
    return fail(c, SQRTBA_E_UNSUPPORTED, "explicit Schur complement with %lld blocks", (long long)sc.noff);
  sc.blk_prob.resize(sc.noff);
  std::vector<int64_t> rc(NC + 1, 0);
  for (int64_t q = 0; q < NC; ++q) rc[q + 1] += 1;  // diagonal
  for (int64_t b = 0; b < sc.noff; ++b) {
    rc[bca[b] + 1]++;
    rc[bcb[b] + 1]++;
    sc.blk_prob[b] = h.cam_prob[bca[b]];
  }
  for (int64_t q = 0; q < NC; ++q) rc[q + 1] += rc[q];
  sc.rowoff.assign(rc.begin(), rc.end());
  sc.rowent.resize(2 * rc[NC]);
  std::vector<int64_t> fill(rc.begin(), rc.end() - 1);
  for (int64_t q = 0; q < NC; ++q) {
    const int64_t f = fill[q]++;
    sc.rowent[2 * f] = (int32_t)(sc.noff + q);
    sc.rowent[2 * f + 1] = (int32_t)q;
  }
  for (int64_t b = 0; b < sc.noff; ++b) {
    int64_t f = fill[bca[b]]++;
    sc.rowent[2 * f] = (int32_t)b;
    sc.rowent[2 * f + 1] = bcb[b];
    f = fill[bcb[b]]++;
    sc.rowent[2 * f] = (int32_t)((uint32_t)b | 0x80000000u);
    sc.rowent[2 * f + 1] = bca[b];
  }
  sc.built = true;
  h.sc = std::move(sc);
  return SQRTBA_OK;
}

uint64_t layout(const HostData& h, int mode, void* base, Dev* d) {
  const bool implicit = mode != 0, sc = mode == 2;
  Layout L;
  const uint64_t NC = h.NC, NL = h.NL, NO = h.NO, NS = h.NS, P = h.P;
  Dev t{};
  auto f32 = [&](uint64_t n) { return L.take(4 * n); };
  auto f64 = [&](uint64_t n) { return L.take(8 * n); };
  auto fr = [&](uint64_t n) { return L.take(sizeof(real) * n); };
  uint64_t o_cam = fr(16 * NC), o_camn = fr(16 * NC), o_pts = fr(4 * NL), o_ptsn = fr(4 * NL);
  uint64_t o_ocam = f32(NO), o_olm = f32(NO), o_ouv = fr(2 * NO), o_coo = f32(NC + 1), o_coi = f32(NO);
  uint64_t o_cpr = f32(NC), o_lpr = f32(NL), o_pco = f32(P + 1), o_plo = f32(P + 1);
  uint64_t o_slm = f32(NS), o_sk = f32(NS), o_so = f32(NS), o_sp = f32(NS), o_sb = f64(NS), o_st = f64(NS);
  uint64_t o_sz = f32(NS), o_czp = f32(NO);
  uint64_t o_lms = f32(NL);
  uint64_t o_qj = f32(h.qjob.size()), o_hj = f32(h.hjob.size()), o_hzo = f64(h.hz_off.size()), o_zp = fr(h.hz_floats);
  const uint64_t nB = implicit ? 0 : h.poolB, nT = implicit ? 0 : h.poolT, nrho = implicit ? 0 : 2 * NO;
  uint64_t o_pB = fr(nB), o_pT = fr(nT), o_lmd = fr(NS * LMD_STRIDE), o_rho = fr(nrho);
  uint64_t o_rec = fr(implicit ? 4 * (uint64_t)REC_PLANES * NO : 0), o_rcam = f32(implicit ? NO : 0);
  uint64_t o_vzs = fr(12 * NC);
  const uint64_t nsb = sc ? (uint64_t)(h.sc.noff + NC) * 81 : 0;
  uint64_t o_scb = fr(nsb), o_scoff = f32(sc ? h.sc.coff.size() : 0), o_scc = f32(sc ? h.sc.contrib.size() : 0);
  uint64_t o_scro = f32(sc ? h.sc.rowoff.size() : 0), o_scre = f32(sc ? h.sc.rowent.size() : 0), o_vy = fr(9 * NC);
  uint64_t o_sc = fr(9 * NC), o_jtj = fr(54 * NC);
  uint64_t o_v[6];
  for (int i = 0; i < 6; ++i) o_v[i] = fr(9 * NC);
  uint64_t o_minv = fr(81 * NC), o_ob = fr(54 * NO), o_dxl = fr(3 * NL), o_tt = fr(implicit ? 0 : 32 * NO);
  uint64_t o_cp = f64(NC), o_cp2 = f64(NC), o_cp3 = f64(NC), o_lp = f64(NL);
  int64_t longest = 1;  // longest per-problem range of landmark or camera partials
  for (int64_t p = 0; p < (int64_t)P; ++p)
    longest = std::max({longest, h.pt_off[p + 1] - h.pt_off[p], h.cam_off[p + 1] - h.cam_off[p]});
  const uint64_t nchunks = (uint64_t)((longest + SUM_CHUNK_VALUES - 1) / SUM_CHUNK_VALUES);
  uint64_t o_psum = f64(P * nchunks);
  uint64_t o_s[10];
  for (int i = 0; i < 10; ++i) o_s[i] = f64(P);
  uint64_t o_it = f32(P), o_dn = f32(P), o_ps = f32(P), o_act = L.take(P), o_flag = L.take(P);
  uint64_t o_cf = f32(4), o_skip = f32(1);
  uint64_t o_csnap = fr(16 * NC), o_psnap = fr(4 * NL);
  uint64_t o_feat = f32(64 * NC), o_lfac = f32(45 * NC), o_cst = f32(4 * NC);
  if (base && d) {
    t.P = (int32_t)P; t.NC = (int32_t)NC; t.NL = (int32_t)NL; t.NS = (int32_t)NS; t.NO = (int32_t)NO;
    t.cam = at<real>(base, o_cam); t.cam_new = at<real>(base, o_camn);
    t.pts = at<real4>(base, o_pts); t.pts_new = at<real4>(base, o_ptsn);
    t.obs_cam = at<int32_t>(base, o_ocam); t.obs_lm = at<int32_t>(base, o_olm); t.obs_uv = at<real2>(base, o_ouv);
    t.cam_obs_off = at<int32_t>(base, o_coo); t.cam_obs_idx = at<int32_t>(base, o_coi);
    t.cam_prob = at<int32_t>(base, o_cpr); t.lm_prob = at<int32_t>(base, o_lpr);
    t.prob_cam_off = at<int32_t>(base, o_pco); t.prob_lm_off = at<int32_t>(base, o_plo);
    t.slot_lm = at<int32_t>(base, o_slm); t.slot_k = at<int32_t>(base, o_sk); t.slot_obs0 = at<int32_t>(base, o_so);
    t.slot_prob = at<int32_t>(base, o_sp); t.slot_boff = at<int64_t>(base, o_sb); t.slot_toff = at<int64_t>(base, o_st);
    t.slot_zoff = at<int32_t>(base, o_sz); t.cam_zpos = at<int32_t>(base, o_czp);
    t.lm_slot = at<int32_t>(base, o_lms);
    t.qjob = at<int2>(base, o_qj); t.hjob = at<int2>(base, o_hj); t.hz_off = at<int64_t>(base, o_hzo); t.zpart = at<real>(base, o_zp);
    t.poolB = at<real>(base, o_pB); t.poolT = at<real>(base, o_pT); t.lmd = at<real>(base, o_lmd);
    t.rhoB = implicit ? nullptr : at<real>(base, o_rho); t.s_cam = at<real>(base, o_sc); t.cam_jtj = at<real>(base, o_jtj);
    if (implicit) { t.poolB = nullptr; t.poolT = nullptr; }
    t.obsrec = implicit ? at<real>(base, o_rec) : nullptr;
    t.rec_cam = implicit ? at<int32_t>(base, o_rcam) : nullptr;
    t.vzs = at<real>(base, o_vzs);
    t.implicit = implicit ? 1 : 0;
    t.sc = sc ? 1 : 0;
    t.sc_noff = sc ? (int32_t)h.sc.noff : 0;
    t.scb = sc ? at<real>(base, o_scb) : nullptr;
    t.sc_coff = sc ? at<int32_t>(base, o_scoff) : nullptr;
    t.sc_contrib = sc ? at<int4>(base, o_scc) : nullptr;
    t.sc_rowoff = sc ? at<int32_t>(base, o_scro) : nullptr;
    t.sc_rowent = sc ? at<int2>(base, o_scre) : nullptr;
    t.vy = at<real>(base, o_vy);
    t.vx = at<real>(base, o_v[0]); t.vr = at<real>(base, o_v[1]); t.vz = at<real>(base, o_v[2]);
    t.vp = at<real>(base, o_v[3]); t.vq = at<real>(base, o_v[4]); t.vb = at<real>(base, o_v[5]);
    t.minv = at<real>(base, o_minv); t.obsbuf = at<real>(base, o_ob); t.dxl = at<real>(base, o_dxl);
    t.ttop = implicit ? nullptr : at<real>(base, o_tt);
    t.cam_part = at<double>(base, o_cp); t.cam_part2 = at<double>(base, o_cp2); t.cam_part3 = at<double>(base, o_cp3);
    t.lm_part = at<double>(base, o_lp);
    t.psum = at<double>(base, o_psum);
    t.sum_chunks = (int32_t)nchunks;
    t.lambda = at<double>(base, o_s[0]); t.rz_next = at<double>(base, o_s[1]); t.beta = at<double>(base, o_s[2]);
    t.rz = at<double>(base, o_s[3]); t.rr = at<double>(base, o_s[4]); t.rr0 = at<double>(base, o_s[5]);
    t.pcost = at<double>(base, o_s[6]); t.ppred = at<double>(base, o_s[7]);
    t.qmod = at<double>(base, o_s[8]); t.dqmod = at<double>(base, o_s[9]);
    t.iters = at<int32_t>(base, o_it); t.done = at<int32_t>(base, o_dn); t.pstatus = at<int32_t>(base, o_ps);
    t.active = at<uint8_t>(base, o_act); t.flag = at<uint8_t>(base, o_flag);
    t.chol_fail = at<int32_t>(base, o_cf);
    t.pcg_skip = at<int32_t>(base, o_skip);
    t.cam_snap = at<real>(base, o_csnap); t.pts_snap = at<real4>(base, o_psnap);
    t.feats = at<float>(base, o_feat); t.lfac = at<float>(base, o_lfac); t.cam_stats = at<float>(base, o_cst);
    *d = t;
  }
  return L.total;
}

hipEvent_t take_event(sqrtba_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Resolve recorded stage events (the stream has been synchronized by the caller).
void flush_profile(sqrtba_ctx* c) {
  for (auto& p : c->pending) {
    float ms = 0.f;
    (void)hipEventSynchronize(p.b);  // stages may return without waiting for the device
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof.ms[p.stage] += ms;
      c->prof.launches[p.stage] += 1;
      c->prof.bytes[p.stage] += p.bytes;
      c->prof.units[p.stage] += p.units;
    } else {
      (void)hipGetLastError();
    }
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
  }
  c->pending.clear();
}

// Run `launches` between two events on the context stream when profiling.
template <typename F>
int timed(sqrtba_ctx* c, int stage, double bytes, int64_t units, F launches) {
  if (!c->prof_on) return launches();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return fail(c, SQRTBA_E_HIP, "hipEventCreate failed");
  HIP_TRY(c, hipEventRecord(a, c->stream));
  const int st = launches();
  HIP_TRY(c, hipEventRecord(b, c->stream));
  c->pending.push_back({stage, a, b, bytes, units});
  return st;
}

double active_sum(const sqrtba_ctx* c, const std::vector<double>& v) {
  double s = 0;
  for (int p = 0; p < c->h.P; ++p)
    if (c->active[p]) s += v[p];
  return s;
}

int64_t active_blocks(const sqrtba_ctx* c) {
  int64_t s = 0;
  for (int p = 0; p < c->h.P; ++p)
    if (c->active[p]) s += c->blocks[p];
  return s;
}

int check_ready(sqrtba_ctx* c) {
  if (c->h.NC < 0 || c->h.NL < 0 || !c->h.obs_set)
    return fail(c, SQRTBA_E_STATE, "set cameras, landmarks and observations first");
  return SQRTBA_OK;
}

template <typename T>
int upload_vec(sqrtba_ctx* c, T* dst, const std::vector<T>& v) {
  if (v.empty()) return SQRTBA_OK;
  HIP_TRY(c, hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return SQRTBA_OK;
}

// Bucket edge and block size of the row-block product: rebuild and upload its
// job list when either changes.
int set_row_blocks(sqrtba_ctx* c, int rows_min_k, int rows) {
  if (rows_min_k == c->L.rows_min_k && rows == c->L.huge_rows) return SQRTBA_OK;
  const int64_t nrows = slots_with_k_at_least(c->h, rows_min_k);
  std::vector<int32_t> jobs;
  build_hjobs(c->h, rows, nrows, jobs);
  if (jobs.size() > c->h.hjob.size()) return fail(c, SQRTBA_E_STATE, "row-block job list exceeds its allocation");
  TRY(upload_vec(c, reinterpret_cast<int32_t*>(c->d.hjob), jobs));
  c->L.rows_n = (int)nrows;
  c->L.hjobs = (int)(jobs.size() / 2);
  c->L.rows_min_k = rows_min_k;
  c->L.huge_rows = rows;
  return SQRTBA_OK;
}

int upload_state(sqrtba_ctx* c) {
  const HostData& h = c->h;
  std::vector<real> cam(16 * h.NC, 0.f), pts(4 * h.NL, 0.f);
  for (int64_t i = 0; i < h.NC; ++i) {
    double w[3] = {h.cams_bal[9 * i], h.cams_bal[9 * i + 1], h.cams_bal[9 * i + 2]}, R[9];
    so3_exp_d(w, R);
    for (int j = 0; j < 9; ++j) cam[16 * i + j] = (real)R[j];
    for (int j = 0; j < 6; ++j) cam[16 * i + 9 + j] = h.cams_bal[9 * i + 3 + j];
  }
  for (int64_t i = 0; i < h.NL; ++i)
    for (int j = 0; j < 3; ++j) pts[4 * i + j] = h.pts[3 * i + j];
  TRY(upload_vec(c, c->d.cam, cam));
  TRY(upload_vec(c, reinterpret_cast<real*>(c->d.pts), pts));
  return SQRTBA_OK;
}

int upload(sqrtba_ctx* c) {
  const HostData& h = c->h;
  Dev& d = c->d;
  layout(h, c->opt.landmark_blocks, c->arena.base, &d);
  d.done_host = c->done_host_dev;
  d.pcg_tol = (real)c->opt.pcg_rel_tol;
  d.pcg_eta = (real)c->opt.pcg_forcing_eta;
  d.huber = (real)c->opt.huber_delta;
  HIP_TRY(c, hipMemsetAsync(c->arena.base, 0, c->arena.bytes, c->stream));
  TRY(upload_state(c));
  TRY(upload_vec(c, d.obs_cam, h.ocam));
  TRY(upload_vec(c, d.obs_lm, h.olm));
  TRY(upload_vec(c, reinterpret_cast<real*>(d.obs_uv), h.ouv));
  TRY(upload_vec(c, d.cam_obs_off, h.cam_obs_off));
  TRY(upload_vec(c, d.cam_obs_idx, h.cam_obs_idx));
  TRY(upload_vec(c, d.cam_prob, h.cam_prob));
  TRY(upload_vec(c, d.lm_prob, h.lm_prob));
  TRY(upload_vec(c, d.prob_cam_off, h.prob_cam_off));
  TRY(upload_vec(c, d.prob_lm_off, h.prob_lm_off));
  TRY(upload_vec(c, d.slot_lm, h.slot_lm));
  TRY(upload_vec(c, d.slot_k, h.slot_k));
  TRY(upload_vec(c, d.slot_obs0, h.slot_obs0));
  TRY(upload_vec(c, d.slot_prob, h.slot_prob));
  TRY(upload_vec(c, d.slot_boff, h.slot_boff));
  TRY(upload_vec(c, d.slot_toff, h.slot_toff));
  if (d.implicit) {
    // records in slot order; the product writes 12 floats (3 float4) per record
    std::vector<int32_t> rec0(h.NS), zpos(h.NO), rcam(h.NO);
    int64_t r = 0;
    for (int64_t s = 0; s < h.NS; ++s) {
      rec0[s] = (int32_t)r;
      r += h.slot_k[s];
    }
    for (int64_t q = 0; q < h.NO; ++q) {
      const int32_t j = h.cam_obs_idx[q], s = h.lm_slot[h.olm[j]];
      const int32_t ri = rec0[s] + (j - h.slot_obs0[s]);
      zpos[q] = 12 * ri;
      rcam[ri] = h.ocam[j];
    }
    TRY(upload_vec(c, d.slot_zoff, rec0));
    TRY(upload_vec(c, d.cam_zpos, zpos));
    TRY(upload_vec(c, d.rec_cam, rcam));
    if (d.sc) {
      TRY(upload_vec(c, d.sc_coff, h.sc.coff));
      TRY(upload_vec(c, reinterpret_cast<int32_t*>(d.sc_contrib), h.sc.contrib));
      TRY(upload_vec(c, d.sc_rowoff, h.sc.rowoff));
      TRY(upload_vec(c, reinterpret_cast<int32_t*>(d.sc_rowent), h.sc.rowent));
    }
  } else {
    TRY(upload_vec(c, d.slot_zoff, h.slot_zoff));
    TRY(upload_vec(c, d.cam_zpos, h.cam_zpos));
  }
  TRY(upload_vec(c, d.lm_slot, h.lm_slot));
  TRY(upload_vec(c, reinterpret_cast<int32_t*>(d.hjob), h.hjob));
  TRY(upload_vec(c, reinterpret_cast<int32_t*>(d.qjob), h.qjob));
  TRY(upload_vec(c, d.hz_off, h.hz_off));
  TRY(upload_vec(c, d.cam_stats, h.cam_stats));
  c->active.assign(h.P, 1);
  d.all_active = 1;
  TRY(upload_vec(c, d.active, c->active));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->L.stream = c->stream;
  for (int i = 0; i < NUM_CLASSES; ++i) c->L.wc[i] = h.wc[i];
  c->L.qjobs = (int)(h.qjob.size() / 2);
  // default launch shapes (the autotuner may replace them): the row-block
  // kernel takes class 5 in 64-row blocks, class 4 stays in the main launch
  // unless it is large
  c->L.n45 = (int)slots_with_k_at_least(h, ROWS_MIN_K);
  c->L.huge_rows = 0;
  c->L.rows_min_k = 0;
  c->L.huge_side = 0;
  c->L.large_sep = h.wc[4].slots >= 256;
  c->L.mv_rbs = 0;
  c->L.persist = 0;
  c->L.nt = 0;
  TRY(set_row_blocks(c, class_kmax(4) + 1, HUGE_ROWS_MIN));
  if (!c->side) {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  c->L.side = c->side;
  c->L.fork = c->ev_fork;
  c->L.join = c->ev_join;
  const size_t need = (size_t)h.P * 8 * PINNED_SLICES + 64;
  if (c->pinned_bytes < need) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    HIP_TRY(c, hipHostMalloc(&c->pinned, need, hipHostMallocDefault));
    c->pinned_bytes = need;
  }
  if (c->done_host_n < h.P) {
    // without coherent mapped host memory the host copies the flags back instead
    if (c->done_host) (void)hipHostFree(c->done_host);
    c->done_host = c->done_host_dev = nullptr;
    c->done_host_n = 0;
    void* hp = nullptr;
    const hipError_t ae =
        hipHostMalloc(&hp, sizeof(int32_t) * std::max<int64_t>(1, h.P), hipHostMallocCoherent | hipHostMallocMapped);
    if (ae == hipSuccess) {
      void* dp = nullptr;
      if (hipHostGetDevicePointer(&dp, hp, 0) == hipSuccess) {
        c->done_host = static_cast<int32_t*>(hp);
        c->done_host_dev = static_cast<int32_t*>(dp);
        c->done_host_n = h.P;
      } else {
        (void)hipGetLastError();  // the refusal leaves no error behind
        (void)hipHostFree(hp);
      }
    } else {
      (void)hipGetLastError();
    }
  }
  c->d.done_host = c->done_host_dev;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  const double RB = sizeof(real);  // bytes per element
  c->mv_bytes.assign(h.P, 0.0);
  c->qr_bytes.assign(h.P, 0.0);
  c->blocks.assign(h.P, 0);
  for (int64_t sl = 0; sl < h.NS; ++sl) {
    const double k = h.slot_k[sl];
    const int p = h.slot_prob[sl];
    if (c->opt.landmark_blocks == 2) {
      // explicit Schur complement: the per-landmark preparation writes the 28-float records
      c->qr_bytes[p] += RB * (28.0 * k + 12.0) + (4.0 + 2.0 * RB) * k + 4.0 * RB;
    } else if (c->opt.landmark_blocks == 1) {
      // implicit: read the 24 Jacobian and Q1 floats and the camera index per
      // observation and the 6 floats of P, write 9k per-observation outputs; the
      // QR writes the 28-float records
      c->mv_bytes[p] += RB * (25.0 * k + 6.0 + 9.0 * k);
      c->qr_bytes[p] += RB * (28.0 * k + 12.0) + (4.0 + 2.0 * RB) * k + 4.0 * RB;
    } else {
      // matvec: read the 2k x 9k B rows, write 9k per-observation outputs
      c->mv_bytes[p] += RB * (18.0 * k * k + 9.0 * k);
      // QR: write 2k rotated rows (9k pose columns + residual) and the 12-float
      // landmark record; read camera index and pixel per observation, the landmark
      c->qr_bytes[p] += RB * (2.0 * k * (9.0 * k + 1.0) + 12.0) + (4.0 + 2.0 * RB) * k + 4.0 * RB;
    }
    c->blocks[p] += 1;
  }
  if (c->opt.landmark_blocks == 2) {
    // product with the reduced matrix: every off-diagonal block is read from both of
    // its cameras' rows, every diagonal block once (81 floats and the 12-float
    // gathered vector each), and 9 outputs per camera are written
    for (int64_t b = 0; b < h.sc.noff; ++b) c->mv_bytes[h.sc.blk_prob[b]] += 2.0 * RB * (81.0 + 12.0);
    for (int64_t q = 0; q < h.NC; ++q) c->mv_bytes[h.cam_prob[q]] += RB * (81.0 + 12.0 + 9.0);
  }
  c->snapshot = false;
  c->uploaded = true;
  c->linearized = c->marginalized = c->damped = c->solved = c->backsubbed = c->updated = false;
  return SQRTBA_OK;
}

void release_arena(sqrtba_ctx* c) {
  if (c->arena.owned && c->arena.base) (void)hipFree(c->arena.base);
  c->arena = Arena{};
  c->uploaded = false;
}

int ensure_uploaded(sqrtba_ctx* c) {
  if (c->uploaded) return SQRTBA_OK;
  TRY(check_ready(c));
  if (c->opt.landmark_blocks == 2) TRY(build_sc(c));
  const uint64_t bytes = layout(c->h, c->opt.landmark_blocks, nullptr, nullptr);
  release_arena(c);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(c, SQRTBA_E_OOM, "hipMalloc(%llu) failed: %s", (unsigned long long)bytes, hipGetErrorString(e));
  c->arena = Arena{p, bytes, true};
  return upload(c);
}

// read back n per-problem values of type T from a device array
template <typename T>
int readback(sqrtba_ctx* c, const T* dev, T* out, bool sync = true) {
  const size_t bytes = sizeof(T) * c->h.P;
  HIP_TRY(c, hipMemcpyAsync(c->pinned, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  if (sync) HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (out) std::memcpy(out, c->pinned, bytes);
  return SQRTBA_OK;
}

// The pinned staging buffer holds PINNED_SLICES slices of 8 bytes per problem:
// slice 0 for readback, slices 0..3 for readback_all, 4 for a deferred copy of
// the model decrease, 5 (PCG iteration counts, then statuses), 8 (r.r) and 9
// (r0.r0) for a deferred copy of a solve's outcome, 6 for the accept mask and 7
// for lambda.
char* pinned_slice(sqrtba_ctx* c, int j) { return static_cast<char*>(c->pinned) + (size_t)8 * c->h.P * j; }

// Several per-problem arrays copied back with one wait (array j to slice j).
struct Readback {
  const void* dev;
  void* out;
  size_t elem;
};
int readback_all(sqrtba_ctx* c, std::initializer_list<Readback> list) {
  const size_t P = c->h.P;
  int j = 0;
  for (const Readback& r : list)
    HIP_TRY(c, hipMemcpyAsync(pinned_slice(c, j++), r.dev, r.elem * P, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  j = 0;
  for (const Readback& r : list) {
    if (r.out) std::memcpy(r.out, pinned_slice(c, j), r.elem * P);
    ++j;
  }
  return SQRTBA_OK;
}

int set_active_mask(sqrtba_ctx* c, const std::vector<uint8_t>& m) {
  c->active = m;
  c->d.all_active = std::all_of(m.begin(), m.end(), [](uint8_t a) { return a != 0; }) ? 1 : 0;
  HIP_TRY(c, hipMemcpyAsync(c->d.active, c->active.data(), c->active.size(), hipMemcpyHostToDevice, c->stream));
  return SQRTBA_OK;
}

#define LAUNCH(ctx, expr)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, SQRTBA_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int do_linearize(sqrtba_ctx* c, double* cost) {
  TRY(ensure_uploaded(c));
  TRY(timed(c, SQRTBA_STAGE_LINEARIZE, 0.0, 0, [&]() {
    LAUNCH(c, launch_cam_linearize(c->d, c->L, true, false, c->d.active));
    LAUNCH(c, launch_prob_sum(c->d, c->L, c->d.cam_part, c->d.prob_cam_off, c->d.pcost, c->d.active));
    return (int)SQRTBA_OK;
  }));
  TRY(readback(c, c->d.pcost, cost));
  flush_profile(c);
  c->linearized = true;
  c->marginalized = c->damped = c->solved = c->backsubbed = c->updated = false;
  return SQRTBA_OK;
}

// sync = false (inside the LM loop): the stage is enqueued and the host goes
// on; the next stage that reads results back waits for it.
int do_marginalize(sqrtba_ctx* c, bool sync = true) {
  TRY(ensure_uploaded(c));
  if (!c->linearized) return fail(c, SQRTBA_E_STATE, "marginalize needs linearize");
  TRY(timed(c, SQRTBA_STAGE_MARGINALIZE, active_sum(c, c->qr_bytes), active_blocks(c), [&]() {
    LAUNCH(c, launch_marginalize(c->d, c->L, c->d.active));
    return (int)SQRTBA_OK;
  }));
  if (sync) HIP_TRY(c, hipStreamSynchronize(c->stream));
  flush_profile(c);
  c->marginalized = true;
  c->damped = c->solved = c->backsubbed = c->updated = false;
  return SQRTBA_OK;
}

int do_damp(sqrtba_ctx* c, const double* lambda, bool sync = true) {
  if (!c->marginalized) return fail(c, SQRTBA_E_STATE, "damp needs marginalize");
  if (!lambda) return fail(c, SQRTBA_E_INVALID, "null lambda");
  for (int32_t p = 0; p < c->h.P; ++p)
    if (c->active[p] && !(lambda[p] > 0.0 && std::isfinite(lambda[p])))
      return fail(c, SQRTBA_E_INVALID, "lambda[%d] = %g must be positive and finite", p, lambda[p]);
  // (the slice is rewritten only by the next damp, after a later stage has waited)
  std::memcpy(pinned_slice(c, 7), lambda, sizeof(double) * c->h.P);
  HIP_TRY(c, hipMemcpyAsync(c->d.lambda, pinned_slice(c, 7), sizeof(double) * c->h.P, hipMemcpyHostToDevice,
                            c->stream));
  TRY(timed(c, SQRTBA_STAGE_DAMP, 0.0, active_blocks(c), [&]() {
    LAUNCH(c, launch_damp(c->d, c->L, c->d.active));
    return (int)SQRTBA_OK;
  }));
  if (sync) HIP_TRY(c, hipStreamSynchronize(c->stream));
  flush_profile(c);
  c->damped = true;
  c->solved = c->backsubbed = c->updated = false;
  return SQRTBA_OK;
}

// One chunk of n PCG iterations, as a captured graph or as plain launches.
// With profiling on, every matvec is bracketed by events and the caller turns
// the first `live` pairs into stage time after synchronizing.
int run_pcg_chunk(sqrtba_ctx* c, int n, std::vector<std::pair<hipEvent_t, hipEvent_t>>* mv_events) {
  const bool prof = c->prof_on;
  auto iteration = [&](hipEvent_t a, hipEvent_t b) -> hipError_t {
    hipError_t e = hipSuccess;
    if (a) e = hipEventRecord(a, c->stream);
    if (e == hipSuccess) e = launch_matvec(c->d, c->L);
    if (e == hipSuccess && b) e = hipEventRecord(b, c->stream);
    if (e == hipSuccess) e = launch_pcg_vector(c->d, c->L);
    return e;
  };
  // with the profiler on, iterations are launched one by one (an event pair
  // around every matvec); the kernels are the same as in the graph
  if (c->opt.use_graph && !prof && n == c->opt.pcg_check_every) {
    if (c->graph && c->graph_profiled != prof) {
      (void)hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
    }
    if (!c->graph) {
      hipGraph_t g = nullptr;
      HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      hipError_t le = hipSuccess;
      for (int i = 0; i < n && le == hipSuccess; ++i) le = iteration(nullptr, nullptr);
      hipError_t ee = hipStreamEndCapture(c->stream, &g);
      if (le != hipSuccess) return fail(c, SQRTBA_E_HIP, "PCG capture: %s", hipGetErrorString(le));
      if (ee != hipSuccess) return fail(c, SQRTBA_E_HIP, "PCG capture end: %s", hipGetErrorString(ee));
      hipError_t ie = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        c->graph = nullptr;
        return fail(c, SQRTBA_E_HIP, "PCG graph instantiate: %s", hipGetErrorString(ie));
      }
      c->graph_iters = n;
      c->graph_profiled = prof;
    }
    HIP_TRY(c, hipGraphLaunch(c->graph, c->stream));
    return SQRTBA_OK;
  }
  for (int i = 0; i < n; ++i) {
    hipEvent_t a = prof ? take_event(c) : nullptr, b = prof ? take_event(c) : nullptr;
    LAUNCH(c, iteration(a, b));
    if (prof && mv_events) mv_events->push_back({a, b});
  }
  return SQRTBA_OK;
}

LearnDev learn_dev(sqrtba_ctx* c) {
  LearnDev m{};
  m.w32 = c->ln.w32;
  m.wbf = c->ln.wbf;
  m.adam_m = c->ln.adam_m;
  m.adam_v = c->ln.adam_v;
  m.feats = c->d.feats;
  m.lfac = c->d.lfac;
  return m;
}

int ensure_learned(sqrtba_ctx* c) {
  auto& L = c->ln;
  if (L.alloc) return SQRTBA_OK;
  const size_t n = MLP_PARAMS;
  HIP_TRY(c, hipMalloc(&L.w32, 4 * n));
  HIP_TRY(c, hipMalloc(&L.wbf, 2 * n));
  HIP_TRY(c, hipMalloc(&L.adam_m, 4 * n));
  HIP_TRY(c, hipMalloc(&L.adam_v, 4 * n));
  HIP_TRY(c, hipMalloc(&L.grad, 4 * n));
  L.alloc = true;
  return SQRTBA_OK;
}

// Xavier-uniform first two layers, zero biases and zero last layer: the initial
// network reproduces plain block-Jacobi exactly.
[[maybe_unused]] int init_params(sqrtba_ctx* c, uint64_t seed) {
  TRY(ensure_learned(c));
  std::vector<float> w(MLP_PARAMS, 0.f);
  std::mt19937_64 rng(seed);
  auto fill = [&](size_t off, int fin, int fout) {
    const double lim = std::sqrt(6.0 / (fin + fout));
    std::uniform_real_distribution<double> u(-lim, lim);
    for (size_t i = 0; i < (size_t)fin * fout; ++i) w[off + i] = (float)u(rng);
  };
  fill(0, MLP_IN, MLP_HIDDEN);
  fill((size_t)MLP_IN * MLP_HIDDEN + MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN);
  HIP_TRY(c, hipMemcpyAsync(c->ln.w32, w.data(), 4 * w.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ln.adam_m, 0, 4 * w.size(), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ln.adam_v, 0, 4 * w.size(), c->stream));
  LAUNCH(c, launch_to_bf16(learn_dev(c), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->ln.adam_step = 0;
  return SQRTBA_OK;
}

// copy p and q of the iteration just launched into the trace store
int trace_iteration(sqrtba_ctx* c) {
  auto& L = c->ln;
  if (L.cur_solve < 0 || L.cur_iter >= L.iters_per_solve) return SQRTBA_OK;
  const size_t N = 9 * (size_t)c->h.NC;
  const int r = L.n_records;
  HIP_TRY(c, hipMemcpyAsync(L.t_p + N * r, c->d.vp, 4 * N, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(L.t_q + N * r, c->d.vq, 4 * N, hipMemcpyDeviceToDevice, c->stream));
  L.h_rec_solve.push_back(L.cur_solve);
  L.n_records++;
  L.cur_iter++;
  return SQRTBA_OK;
}

// Where the convergence test runs (sqrtba_options::pcg_test_kernel): its own
// kernel when the product it saves once per solve outweighs one small launch
// per iteration, i.e. when the product moves at least 1 GiB.
int pcg_test_sep(const sqrtba_ctx* c) {
  if (c->opt.pcg_test_kernel >= 0) return c->opt.pcg_test_kernel;
  double b = 0.0;
  for (int p = 0; p < c->h.P; ++p)
    if (c->active[p]) b += c->mv_bytes[p];
  return b >= 1073741824.0 ? 1 : 0;
}

// PCG on the current minv blocks from x0 = 0, at most cap iterations.
int run_pcg(sqrtba_ctx* c, int cap) {
  const int P = c->h.P;
  const int ts = pcg_test_sep(c);
  if (ts != c->d.test_sep) {
    c->d.test_sep = ts;
    if (c->graph) {  // captured launches hold the old Dev values
      (void)hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
    }
  }
  LAUNCH(c, launch_pcg_init(c->d, c->L));
  std::vector<int32_t> done(P);
  if (c->done_host) {
    // no wait here: every active problem counts as running until the first
    // chunk's flags arrive (a problem the start kernels found done, e.g. with a
    // zero right-hand side, costs one chunk whose kernels exit at once).  The
    // kernels of this solve overwrite every flag before the host reads it;
    // until then a stale value can only be 0 (one more chunk).
    for (int p = 0; p < P; ++p) done[p] = c->active[p] ? 0 : 1;
    std::memset(c->done_host, 0, sizeof(int32_t) * P);
  } else {
    TRY(readback(c, c->d.done, done.data()));
  }
  auto all_done = [&]() {
    for (int p = 0; p < P; ++p)
      if (!done[p]) return false;
    return true;
  };
  int it = 0;
  const bool tracing = c->ln.cur_solve >= 0;
  const int every = std::max(1, c->opt.pcg_check_every);
  std::vector<int32_t> its_before(P, 0), its_after(P, 0);
  std::vector<std::pair<hipEvent_t, hipEvent_t>> mv;
  while (it < cap && !all_done()) {
    const int n = std::min(every, cap - it);
    mv.clear();
    if (tracing) {
      for (int i = 0; i < n; ++i) {
        hipEvent_t a = c->prof_on ? take_event(c) : nullptr, b = c->prof_on ? take_event(c) : nullptr;
        if (a) HIP_TRY(c, hipEventRecord(a, c->stream));
        LAUNCH(c, launch_matvec(c->d, c->L));
        if (b) HIP_TRY(c, hipEventRecord(b, c->stream));
        LAUNCH(c, launch_pcg_vector(c->d, c->L));
        TRY(trace_iteration(c));
        if (a) mv.push_back({a, b});
      }
    } else {
      TRY(run_pcg_chunk(c, n, &mv));
    }
    it += n;
    if (c->done_host) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      std::memcpy(done.data(), c->done_host, sizeof(int32_t) * P);
    } else {
      TRY(readback(c, c->d.done, done.data()));
    }
    if (c->prof_on) {
      // matvecs of iterations that did work; later ones in the chunk exit at once
      TRY(readback(c, c->d.iters, its_after.data()));
      int live = 0;
      double bytes = 0.0;
      int64_t units = 0;
      for (int p = 0; p < P; ++p) {
        const int di = its_after[p] - its_before[p];
        live = std::max(live, di);
        bytes += c->mv_bytes[p] * di;
        units += c->blocks[p] * di;
      }
      double ms_sum = 0.0;
      for (int i = 0; i < (int)mv.size(); ++i) {
        float ms = 0.f;
        if (i < live) {
          if (hipEventElapsedTime(&ms, mv[i].first, mv[i].second) == hipSuccess)
            ms_sum += ms;
          else
            (void)hipGetLastError();
        }
        c->event_pool.push_back(mv[i].first);
        c->event_pool.push_back(mv[i].second);
      }
      c->prof.ms[SQRTBA_STAGE_MATVEC] += ms_sum;
      c->prof.launches[SQRTBA_STAGE_MATVEC] += live;
      c->prof.bytes[SQRTBA_STAGE_MATVEC] += bytes;
      c->prof.units[SQRTBA_STAGE_MATVEC] += units;
      its_before = its_after;
    }
  }
  LAUNCH(c, launch_pcg_final(c->d, c->L));
  return SQRTBA_OK;
}

int precond_stage(sqrtba_ctx* c) {
  return timed(c, SQRTBA_STAGE_PRECOND, 0.0, active_blocks(c), [&]() {
    LAUNCH(c, launch_precond_rhs(c->d, c->L));
    return (int)SQRTBA_OK;
  });
}

// The per-problem outputs of a solve from its outcome arrays (and, after a
// learned run with fallbacks, the kept problems' outcomes of the learned run).
void finish_solve(sqrtba_ctx* c, bool learned, const std::vector<uint8_t>& fell_back, std::vector<int32_t>& its,
                  std::vector<int32_t>& st, std::vector<double>& rr, std::vector<double>& rr0,
                  const std::vector<int32_t>& kept_its, const std::vector<int32_t>& kept_st,
                  const std::vector<double>& kept_rr, const std::vector<double>& kept_rr0, int32_t* iters,
                  double* rel_res, int32_t* status) {
  const int P = c->h.P;
  auto& L = c->ln;
  if (!kept_its.empty())
    for (int p = 0; p < P; ++p)
      if (c->active[p] && !fell_back[p]) {
        its[p] = kept_its[p];
        st[p] = kept_st[p];
        rr[p] = kept_rr[p];
        rr0[p] = kept_rr0[p];
      }
  for (int p = 0; p < P; ++p) {
    if (c->active[p] && (!learned || fell_back[p])) {
      L.last_plain_iters[p] = its[p];
      L.last_plain_status[p] = st[p];
    }
    if (iters) iters[p] = its[p];
    if (status) status[p] = st[p];
    if (rel_res) rel_res[p] = rr0[p] > 0 ? std::sqrt(std::max(rr[p], 0.0) / rr0[p]) : 0.0;
  }
}

// sync = false (inside the LM loop, plain block-Jacobi only): the outcome
// arrays are copied to pinned slices 5, 8 and 9 without a wait, and
// collect_solve turns them into the outputs after the caller's next wait.
int do_solve(sqrtba_ctx* c, int32_t* iters, double* rel_res, int32_t* status, bool sync = true) {
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "solve needs damp");
  const int P = c->h.P;
  auto& L = c->ln;
  if ((int)L.last_plain_iters.size() != P) L.last_plain_iters.assign(P, -1);
  if ((int)L.last_plain_status.size() != P) L.last_plain_status.assign(P, -1);
  TRY(precond_stage(c));
  // trace store: features and factors of this solve
  L.cur_solve = -1;
  L.cur_iter = 0;
  if (L.max_solves > 0 && L.n_solves < L.max_solves) {
    const size_t NC = c->h.NC;
    HIP_TRY(c, hipMemcpyAsync(L.t_feat + 64 * NC * L.n_solves, c->d.feats, 4 * 64 * NC, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(L.t_lfac + 45 * NC * L.n_solves, c->d.lfac, 4 * 45 * NC, hipMemcpyDeviceToDevice, c->stream));
    L.cur_solve = L.n_solves++;
  }
  const bool learned = L.mode == 1 && L.alloc;
  std::vector<int32_t> its(P), st(P), kept_its, kept_st;
  std::vector<double> kept_rr, kept_rr0;
  std::vector<uint8_t> fell_back(P, 0);
  if (learned) {
    LAUNCH(c, launch_mlp_precond(c->d, learn_dev(c), c->stream));
    int cap = c->opt.pcg_max_iters;
    bool have_all = true;
    int mx = 0;
    for (int p = 0; p < P; ++p)
      if (c->active[p]) {
        if (L.last_plain_iters[p] < 0) have_all = false;
        mx = std::max(mx, L.last_plain_iters[p]);
      }
    if (have_all) cap = std::min(cap, std::max(1, (3 * mx + 1) / 2));
    TRY(run_pcg(c, cap));
    TRY(readback(c, c->d.iters, its.data()));
    TRY(readback(c, c->d.pstatus, st.data()));
    L.learned_solves++;
    // fallback: problems the learned blocks did not bring to the tolerance.
    // A learned run that used the full iteration budget is kept when the
    // last plain run of that problem also ended at the budget: a restart
    // could not reach the tolerance either.
    std::vector<uint8_t> fb(P, 0), keep = c->active;
    bool any = false;
    for (int p = 0; p < P; ++p) {
      if (!c->active[p] || st[p] == SQRTBA_PCG_CONVERGED || st[p] == SQRTBA_PCG_ZERO_RHS) continue;
      const bool budget = st[p] == SQRTBA_PCG_MAX_ITERS && its[p] >= c->opt.pcg_max_iters &&
                          L.last_plain_status[p] == SQRTBA_PCG_MAX_ITERS;
      if (!budget) {
        fb[p] = 1;
        any = true;
        L.fallbacks++;
        L.wasted_iters += its[p];
      }
    }
    if (any) {
      // the restart runs only the fallback problems; the PCG start kernels reset
      // the scalars of every other problem (their x is kept), so the kept
      // problems' outcomes of the learned run are saved and merged back below
      kept_rr.resize(P);
      kept_rr0.resize(P);
      TRY(readback(c, c->d.rr, kept_rr.data()));
      TRY(readback(c, c->d.rr0, kept_rr0.data()));
      kept_its = its;
      kept_st = st;
      TRY(set_active_mask(c, fb));
      TRY(precond_stage(c));  // plain block-Jacobi blocks for these problems
      TRY(run_pcg(c, c->opt.pcg_max_iters));
      TRY(set_active_mask(c, keep));
    }
    fell_back = fb;
  } else {
    TRY(run_pcg(c, c->opt.pcg_max_iters));
  }
  L.cur_solve = -1;
  c->solved = true;
  c->backsubbed = c->updated = false;
  if (!sync && !learned) {
    const size_t P4 = sizeof(int32_t) * P, P8 = sizeof(double) * P;
    HIP_TRY(c, hipMemcpyAsync(pinned_slice(c, 5), c->d.iters, P4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(pinned_slice(c, 5) + P4, c->d.pstatus, P4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(pinned_slice(c, 8), c->d.rr, P8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(pinned_slice(c, 9), c->d.rr0, P8, hipMemcpyDeviceToHost, c->stream));
    c->solve_pending = true;
    flush_profile(c);
    return SQRTBA_OK;
  }
  std::vector<double> rr(P), rr0(P);
  TRY(readback_all(c, {{c->d.iters, its.data(), sizeof(int32_t)}, {c->d.pstatus, st.data(), sizeof(int32_t)},
                       {c->d.rr, rr.data(), sizeof(double)}, {c->d.rr0, rr0.data(), sizeof(double)}}));
  flush_profile(c);
  finish_solve(c, learned, fell_back, its, st, rr, rr0, kept_its, kept_st, kept_rr, kept_rr0, iters, rel_res,
               status);
  return SQRTBA_OK;
}

// The outputs of a solve enqueued with sync = false; the stream must have been
// waited for since (do_update waits).
int collect_solve(sqrtba_ctx* c, int32_t* iters, double* rel_res, int32_t* status) {
  const int P = c->h.P;
  const size_t P4 = sizeof(int32_t) * P, P8 = sizeof(double) * P;
  std::vector<int32_t> its(P), st(P);
  std::vector<double> rr(P), rr0(P);
  std::memcpy(its.data(), pinned_slice(c, 5), P4);
  std::memcpy(st.data(), pinned_slice(c, 5) + P4, P4);
  std::memcpy(rr.data(), pinned_slice(c, 8), P8);
  std::memcpy(rr0.data(), pinned_slice(c, 9), P8);
  c->solve_pending = false;
  finish_solve(c, false, std::vector<uint8_t>(P, 0), its, st, rr, rr0, {}, {}, {}, {}, iters, rel_res, status);
  return SQRTBA_OK;
}

// sync = false: the model decrease is copied to pinned slice 4 without a wait;
// the caller takes it from there after the next wait (do_update's).
int do_backsub(sqrtba_ctx* c, double* pred, bool sync = true) {
  if (!c->solved) return fail(c, SQRTBA_E_STATE, "back_substitute needs solve");
  TRY(timed(c, SQRTBA_STAGE_BACKSUB, 0.0, active_blocks(c), [&]() {
    LAUNCH(c, launch_backsub(c->d, c->L));
    LAUNCH(c, launch_prob_sum(c->d, c->L, c->d.lm_part, c->d.prob_lm_off, c->d.ppred, c->d.active));
    return (int)SQRTBA_OK;
  }));
  if (sync) {
    TRY(readback(c, c->d.ppred, pred));
  } else {
    HIP_TRY(c, hipMemcpyAsync(pinned_slice(c, 4), c->d.ppred, sizeof(double) * c->h.P, hipMemcpyDeviceToHost,
                              c->stream));
  }
  flush_profile(c);
  c->backsubbed = true;
  c->updated = false;
  return SQRTBA_OK;
}

int do_update(sqrtba_ctx* c, double* new_cost) {
  if (!c->backsubbed) return fail(c, SQRTBA_E_STATE, "update needs back_substitute");
  TRY(timed(c, SQRTBA_STAGE_UPDATE, 0.0, 0, [&]() {
    LAUNCH(c, launch_update(c->d, c->L));
    LAUNCH(c, launch_cam_linearize(c->d, c->L, false, true, c->d.active));
    LAUNCH(c, launch_prob_sum(c->d, c->L, c->d.cam_part, c->d.prob_cam_off, c->d.pcost, c->d.active));
    return (int)SQRTBA_OK;
  }));
  TRY(readback(c, c->d.pcost, new_cost));
  flush_profile(c);
  c->updated = true;
  return SQRTBA_OK;
}

int do_commit(sqrtba_ctx* c, const uint8_t* accept, bool sync = true) {
  if (!c->updated) return fail(c, SQRTBA_E_STATE, "commit needs update");
  if (!accept) return fail(c, SQRTBA_E_INVALID, "null accept mask");
  // (the slice is rewritten only by the next commit, after later stages have waited)
  std::memcpy(pinned_slice(c, 6), accept, c->h.P);
  HIP_TRY(c, hipMemcpyAsync(c->d.flag, pinned_slice(c, 6), c->h.P, hipMemcpyHostToDevice, c->stream));
  LAUNCH(c, launch_commit(c->d, c->L));
  if (sync) HIP_TRY(c, hipStreamSynchronize(c->stream));
  bool any = false;
  for (int p = 0; p < c->h.P; ++p) any |= (c->active[p] && accept[p]);
  c->updated = false;
  if (any) c->linearized = c->marginalized = c->damped = c->solved = c->backsubbed = false;
  return SQRTBA_OK;
}

int lm_loop(sqrtba_ctx* c, const double* tol_cost, sqrtba_lm_report* rep) {
  TRY(ensure_uploaded(c));
  const int P = c->h.P;
  const sqrtba_options& o = c->opt;
  c->history.assign(P, {});
  std::vector<uint8_t> all(P, 1), fin(P, 0), acc(P, 0), relin(P, 0);
  std::vector<double> E(P), Enew(P), pred(P), lam(P, o.lambda0), nu(P, 2.0), rel(P), t_tol(P, -1.0), t_fin(P, 0.0);
  std::vector<int32_t> its(P), st(P), lm_it(P, 0), nacc(P, 0), tot_pcg(P, 0), lm_status(P, SQRTBA_LM_MAX_ITERS);
  const double t0 = now_s();
  TRY(set_active_mask(c, all));
  TRY(do_linearize(c, E.data()));
  TRY(do_marginalize(c, false));
  std::vector<double> E0 = E;
  for (int p = 0; p < P; ++p) {
    if (!std::isfinite(E[p])) { fin[p] = 1; lm_status[p] = SQRTBA_LM_NONFINITE; }
    if (tol_cost && E[p] <= tol_cost[p]) t_tol[p] = 0.0;
    if (o.max_lm_iters <= 0) fin[p] = 1;
  }
  while (true) {
    std::vector<uint8_t> act(P);
    bool any = false;
    for (int p = 0; p < P; ++p) { act[p] = !fin[p]; any |= act[p]; }
    if (!any) break;
    TRY(set_active_mask(c, act));
    TRY(do_damp(c, lam.data(), false));
    TRY(do_solve(c, its.data(), rel.data(), st.data(), false));
    TRY(do_backsub(c, nullptr, false));
    TRY(do_update(c, Enew.data()));  // waits, so the model decrease is in slice 4 too
    std::memcpy(pred.data(), pinned_slice(c, 4), sizeof(double) * P);
    if (c->solve_pending) TRY(collect_solve(c, its.data(), rel.data(), st.data()));
    for (int p = 0; p < P; ++p) {
      acc[p] = 0;
      if (!act[p]) continue;
      const double rho = pred[p] > 0 ? (E[p] - Enew[p]) / pred[p] : -INFINITY;
      acc[p] = std::isfinite(Enew[p]) && rho > o.accept_ratio;
    }
    TRY(do_commit(c, acc.data(), false));
    const double tnow = now_s() - t0;
    bool any_relin = false;
    for (int p = 0; p < P; ++p) {
      relin[p] = 0;
      if (!act[p]) continue;
      const double rho = pred[p] > 0 ? (E[p] - Enew[p]) / pred[p] : -INFINITY;
      sqrtba_lm_record r{lm_it[p], acc[p], its[p], st[p], lam[p], E[p], Enew[p], pred[p], rel[p], tnow};
      c->history[p].push_back(r);
      lm_it[p]++;
      tot_pcg[p] += its[p];
      if (acc[p]) {
        nacc[p]++;
        const double rel_dec = (E[p] - Enew[p]) / E[p];
        E[p] = Enew[p];
        const double q = 2.0 * rho - 1.0;
        lam[p] = std::min(std::max(lam[p] * std::max(1.0 / 3.0, 1.0 - q * q * q), o.lambda_min), o.lambda_max);
        nu[p] = 2.0;
        if (tol_cost && t_tol[p] < 0 && E[p] <= tol_cost[p]) t_tol[p] = tnow;
        if (rel_dec < o.func_tol) { fin[p] = 1; lm_status[p] = SQRTBA_LM_FUNC_TOL; }
        else relin[p] = 1;
      } else {
        lam[p] *= nu[p];
        nu[p] *= 2.0;
        if (lam[p] >= o.lambda_max) { fin[p] = 1; lm_status[p] = SQRTBA_LM_LAMBDA_MAX; }
        lam[p] = std::max(lam[p], o.lambda_min);
      }
      if (!fin[p] && lm_it[p] >= o.max_lm_iters) { fin[p] = 1; lm_status[p] = SQRTBA_LM_MAX_ITERS; }
      if (fin[p]) { relin[p] = 0; t_fin[p] = tnow; }
      any_relin |= relin[p];
    }
    if (any_relin) {
      std::vector<double> Er(P);
      TRY(set_active_mask(c, relin));
      TRY(do_linearize(c, Er.data()));
      TRY(do_marginalize(c, false));
      for (int p = 0; p < P; ++p)
        if (relin[p]) E[p] = Er[p];
    }
    // problems that did not relinearize keep their blocks (marginalized) for re-damping
    c->marginalized = true;
    c->linearized = true;
  }
  TRY(set_active_mask(c, all));
  if (rep)
    for (int p = 0; p < P; ++p) {
      rep[p].initial_cost = E0[p];
      rep[p].final_cost = E[p];
      rep[p].iterations = lm_it[p];
      rep[p].accepted = nacc[p];
      rep[p].total_pcg_iters = tot_pcg[p];
      rep[p].status = lm_status[p];
      rep[p].solve_seconds = t_fin[p];
      rep[p].time_to_tol = t_tol[p];
    }
  return SQRTBA_OK;
}

// caller-owned device arrays: checked, then copied over on the context's stream
int32_t check_device_ptr(sqrtba_ctx* c, const void* p, const char* what) {
  if (!p) return fail(c, SQRTBA_E_INVALID, "%s: null pointer", what);
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SQRTBA_E_INVALID, "%s is not a device pointer", what);
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(c, SQRTBA_E_INVALID, "%s is not a device pointer", what);
  return SQRTBA_OK;
}

template <class T>
int32_t from_device(sqrtba_ctx* c, const T* p, int64_t n, std::vector<T>& out, const char* what) {
  TRY(check_device_ptr(c, p, what));
  out.resize((size_t)n);
  HIP_TRY(c, hipMemcpyAsync(out.data(), p, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

template <class T>
int32_t to_device(sqrtba_ctx* c, T* p, const std::vector<T>& in, const char* what) {
  TRY(check_device_ptr(c, p, what));
  HIP_TRY(c, hipMemcpyAsync(p, in.data(), sizeof(T) * in.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

}  // namespace

// ================================================================= C ABI

extern "C" {

int32_t SQRTBA_API(version)(void) { return kVersion; }

void SQRTBA_API(default_options)(sqrtba_options* o) {
  if (!o) return;
  o->lambda0 = 1e-4;
  o->lambda_min = 1e-16;
  o->lambda_max = 1e32;
  o->accept_ratio = 1e-3;
  o->max_lm_iters = 50;
  o->func_tol = 1e-6;
  o->pcg_max_iters = 500;
  o->pcg_rel_tol = 1e-6;
  o->pcg_check_every = 8;
  o->use_graph = 1;
  o->pcg_forcing_eta = 0.0;
  o->landmark_blocks = 0;
  o->huber_delta = 0.0;
  o->pcg_test_kernel = -1;
}

static bool valid_options(const sqrtba_options& o) {
  return o.pcg_max_iters >= 0 && o.max_lm_iters >= 0 && o.lambda0 > 0 && o.pcg_check_every >= 1 &&
         std::isfinite(o.pcg_forcing_eta) && o.pcg_forcing_eta >= 0.0 &&
         (o.landmark_blocks >= 0 && o.landmark_blocks <= 2) && std::isfinite(o.huber_delta) &&
         o.huber_delta >= 0.0 && o.pcg_test_kernel >= -1 && o.pcg_test_kernel <= 1;
}

int32_t SQRTBA_API(create)(sqrtba_ctx** out, const sqrtba_options* opt, void* hip_stream) {
  if (!out) return SQRTBA_E_INVALID;
  *out = nullptr;
  sqrtba_ctx* c = new (std::nothrow) sqrtba_ctx();
  if (!c) return SQRTBA_E_OOM;
  SQRTBA_API(default_options)(&c->opt);
  if (opt) c->opt = *opt;
  if (!valid_options(c->opt)) {
    delete c;
    return SQRTBA_E_INVALID;
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return SQRTBA_E_HIP;
  }
  // the no-allocation product's scratch on this device (looked up once per device)
  if (noalloc_scratch(c->device, &c->noalloc_scratch) != hipSuccess) {
    delete c;
    return SQRTBA_E_HIP;
  }
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return SQRTBA_E_HIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(set_options)(sqrtba_ctx* c, const sqrtba_options* opt) {
  if (!c || !opt || !valid_options(*opt)) return SQRTBA_E_INVALID;
  if (opt->landmark_blocks != c->opt.landmark_blocks && (c->uploaded || c->arena.base))
    return fail(c, SQRTBA_E_STATE, "landmark_blocks is chosen before the workspace is bound");
  if (opt->landmark_blocks == 2 && c->h.obs_set) TRY(build_sc(c));
  c->opt = *opt;
  c->d.pcg_tol = (real)c->opt.pcg_rel_tol;
  c->d.pcg_eta = (real)c->opt.pcg_forcing_eta;
  c->d.huber = (real)c->opt.huber_delta;
  if (c->graph) {  // captured launches hold the old Dev values
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SQRTBA_OK;
}

void SQRTBA_API(destroy)(sqrtba_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  {
    auto& L = c->ln;
    for (void* p : {(void*)L.w32, (void*)L.wbf, (void*)L.adam_m, (void*)L.adam_v, (void*)L.grad, (void*)L.part,
                    (void*)L.loss_part, (void*)L.t_feat, (void*)L.t_lfac, (void*)L.t_p, (void*)L.t_q,
                    (void*)L.rec_solve, (void*)L.s_rec, (void*)L.s_cam})
      if (p) (void)hipFree(p);
  }
  release_arena(c);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->done_host) (void)hipHostFree(c->done_host);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* SQRTBA_API(last_error)(const sqrtba_ctx* c) { return c ? c->err.c_str() : "null context"; }

int32_t SQRTBA_API(set_problems)(sqrtba_ctx* c, int32_t n, const int64_t* cam_off, const int64_t* pt_off) {
  if (!c) return SQRTBA_E_INVALID;
  if (c->h.NC >= 0 || c->h.NL >= 0) return fail(c, SQRTBA_E_STATE, "set_problems must precede set_cameras/set_landmarks");
  if (n <= 0 || !cam_off || !pt_off) return fail(c, SQRTBA_E_INVALID, "need n_problems > 0 and offsets");
  if (cam_off[0] != 0 || pt_off[0] != 0) return fail(c, SQRTBA_E_INVALID, "offsets must start at 0");
  for (int32_t i = 0; i < n; ++i)
    if (cam_off[i + 1] < cam_off[i] || pt_off[i + 1] < pt_off[i]) return fail(c, SQRTBA_E_INVALID, "offsets must not decrease");
  c->h.P = n;
  c->h.cam_off.assign(cam_off, cam_off + n + 1);
  c->h.pt_off.assign(pt_off, pt_off + n + 1);
  c->h.problems_set = true;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(set_cameras)(sqrtba_ctx* c, int64_t n, const real* params) {
  if (!c) return SQRTBA_E_INVALID;
  if (n <= 0 || !params) return fail(c, SQRTBA_E_INVALID, "need n_cams > 0 and parameters");
  if (c->h.problems_set && c->h.cam_off.back() != n) return fail(c, SQRTBA_E_INVALID, "n_cams does not match the problem offsets");
  if (c->h.obs_set && n != c->h.NC) return fail(c, SQRTBA_E_STATE, "camera count cannot change after set_observations");
  for (int64_t i = 0; i < 9 * n; ++i)
    if (!std::isfinite(params[i])) return fail(c, SQRTBA_E_NONFINITE, "camera parameter %lld is not finite", (long long)i);
  c->h.NC = n;
  c->h.cams_bal.assign(params, params + 9 * n);
  if (!c->h.problems_set) c->h.cam_off = {0, n};
  if (c->uploaded) {
    TRY(upload_state(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->linearized = c->marginalized = c->damped = c->solved = c->backsubbed = c->updated = false;
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(set_landmarks)(sqrtba_ctx* c, int64_t n, const real* xyz) {
  if (!c) return SQRTBA_E_INVALID;
  if (n <= 0 || !xyz) return fail(c, SQRTBA_E_INVALID, "need n_points > 0 and coordinates");
  if (c->h.problems_set && c->h.pt_off.back() != n) return fail(c, SQRTBA_E_INVALID, "n_points does not match the problem offsets");
  if (c->h.obs_set && n != c->h.NL) return fail(c, SQRTBA_E_STATE, "landmark count cannot change after set_observations");
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) return fail(c, SQRTBA_E_NONFINITE, "landmark coordinate %lld is not finite", (long long)i);
  c->h.NL = n;
  c->h.pts.assign(xyz, xyz + 3 * n);
  if (!c->h.problems_set) c->h.pt_off = {0, n};
  if (c->uploaded) {
    TRY(upload_state(c));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->linearized = c->marginalized = c->damped = c->solved = c->backsubbed = c->updated = false;
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(set_observations)(sqrtba_ctx* c, int64_t n, const int32_t* cam, const int32_t* pt, const real* uv) {
  if (!c) return SQRTBA_E_INVALID;
  if (c->h.NC < 0 || c->h.NL < 0) return fail(c, SQRTBA_E_STATE, "set cameras and landmarks first");
  TRY(build_bookkeeping(c, n, cam, pt, uv));
  release_arena(c);
  return SQRTBA_OK;
}

int32_t SQRTBA_API(workspace_bytes)(const sqrtba_ctx* c, uint64_t* bytes) {
  if (!c || !bytes) return SQRTBA_E_INVALID;
  if (c->h.NC < 0 || c->h.NL < 0 || !c->h.obs_set) return SQRTBA_E_STATE;
  if (c->opt.landmark_blocks == 2 && !c->h.sc.built) return SQRTBA_E_STATE;
  *bytes = layout(c->h, c->opt.landmark_blocks, nullptr, nullptr);
  return SQRTBA_OK;
}

int32_t SQRTBA_API(bind_workspace)(sqrtba_ctx* c, void* ptr, uint64_t bytes) {
  if (!c) return SQRTBA_E_INVALID;
  TRY(check_ready(c));
  if (c->opt.landmark_blocks == 2) TRY(build_sc(c));
  const uint64_t need = layout(c->h, c->opt.landmark_blocks, nullptr, nullptr);
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return fail(c, SQRTBA_E_INVALID, "workspace must be a 256-byte aligned device pointer");
  if (bytes < need) return fail(c, SQRTBA_E_OOM, "workspace has %llu bytes, needs %llu", (unsigned long long)bytes, (unsigned long long)need);
  release_arena(c);
  c->arena = Arena{ptr, bytes, false};
  return upload(c);
}

int32_t SQRTBA_API(set_active)(sqrtba_ctx* c, const uint8_t* mask) {
  if (!c || !mask) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  std::vector<uint8_t> m(mask, mask + c->h.P);
  for (auto& v : m) v = v ? 1 : 0;
  TRY(set_active_mask(c, m));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(linearize)(sqrtba_ctx* c, double* cost) {
  if (!c) return SQRTBA_E_INVALID;
  return do_linearize(c, cost);
}
int32_t SQRTBA_API(marginalize)(sqrtba_ctx* c) { return c ? do_marginalize(c) : SQRTBA_E_INVALID; }
int32_t SQRTBA_API(damp)(sqrtba_ctx* c, const double* lambda) { return c ? do_damp(c, lambda) : SQRTBA_E_INVALID; }
int32_t SQRTBA_API(solve)(sqrtba_ctx* c, int32_t* iters, double* rel_res, int32_t* status) {
  return c ? do_solve(c, iters, rel_res, status) : SQRTBA_E_INVALID;
}
int32_t SQRTBA_API(back_substitute)(sqrtba_ctx* c, double* pred) { return c ? do_backsub(c, pred) : SQRTBA_E_INVALID; }
int32_t SQRTBA_API(update)(sqrtba_ctx* c, double* new_cost) { return c ? do_update(c, new_cost) : SQRTBA_E_INVALID; }
int32_t SQRTBA_API(commit)(sqrtba_ctx* c, const uint8_t* accept) { return c ? do_commit(c, accept) : SQRTBA_E_INVALID; }
int32_t SQRTBA_API(lm_solve)(sqrtba_ctx* c, sqrtba_lm_report* rep) { return c ? lm_loop(c, nullptr, rep) : SQRTBA_E_INVALID; }
int32_t SQRTBA_API(lm_solve_tracked)(sqrtba_ctx* c, const double* tol, sqrtba_lm_report* rep) {
  return c ? lm_loop(c, tol, rep) : SQRTBA_E_INVALID;
}

int32_t SQRTBA_API(get_lm_history)(const sqrtba_ctx* c, int32_t problem, sqrtba_lm_record* out, int32_t cap, int32_t* n) {
  if (!c || !n) return SQRTBA_E_INVALID;
  if (problem < 0 || problem >= (int32_t)c->history.size()) return SQRTBA_E_INVALID;
  const auto& h = c->history[problem];
  *n = (int32_t)h.size();
  if (out)
    for (int32_t i = 0; i < std::min(cap, *n); ++i) out[i] = h[i];
  return SQRTBA_OK;
}

int32_t SQRTBA_API(get_cameras)(sqrtba_ctx* c, real* params) {
  if (!c || !params) return SQRTBA_E_INVALID;
  if (!c->uploaded) {
    if (c->h.NC < 0) return fail(c, SQRTBA_E_STATE, "no cameras");
    std::memcpy(params, c->h.cams_bal.data(), sizeof(real) * c->h.cams_bal.size());
    return SQRTBA_OK;
  }
  std::vector<real> cam(16 * c->h.NC);
  HIP_TRY(c, hipMemcpyAsync(cam.data(), c->d.cam, cam.size() * sizeof(real), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int64_t i = 0; i < c->h.NC; ++i) {
    double R[9], w[3];
    for (int j = 0; j < 9; ++j) R[j] = cam[16 * i + j];
    so3_log_d(R, w);
    for (int j = 0; j < 3; ++j) params[9 * i + j] = (real)w[j];
    for (int j = 0; j < 6; ++j) params[9 * i + 3 + j] = cam[16 * i + 9 + j];
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(get_landmarks)(sqrtba_ctx* c, real* xyz) {
  if (!c || !xyz) return SQRTBA_E_INVALID;
  if (!c->uploaded) {
    if (c->h.NL < 0) return fail(c, SQRTBA_E_STATE, "no landmarks");
    std::memcpy(xyz, c->h.pts.data(), sizeof(real) * c->h.pts.size());
    return SQRTBA_OK;
  }
  std::vector<real> p(4 * c->h.NL);
  HIP_TRY(c, hipMemcpyAsync(p.data(), c->d.pts, p.size() * sizeof(real), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int64_t i = 0; i < c->h.NL; ++i)
    for (int j = 0; j < 3; ++j) xyz[3 * i + j] = p[4 * i + j];
  return SQRTBA_OK;
}

// ---- device-resident inputs and outputs: the same calls on caller-owned device arrays.
// The bookkeeping (sort by landmark and camera, CSR, size classes) and the rotation
// conversion run on the host, so the arrays are copied over on the context's stream.


int32_t SQRTBA_API(set_cameras_device)(sqrtba_ctx* c, int64_t n, const real* params) {
  if (!c) return SQRTBA_E_INVALID;
  if (n <= 0) return fail(c, SQRTBA_E_INVALID, "need n_cams > 0 and parameters");
  std::vector<real> h;
  TRY(from_device(c, params, 9 * n, h, "camera parameters"));
  return SQRTBA_API(set_cameras)(c, n, h.data());
}

int32_t SQRTBA_API(set_landmarks_device)(sqrtba_ctx* c, int64_t n, const real* xyz) {
  if (!c) return SQRTBA_E_INVALID;
  if (n <= 0) return fail(c, SQRTBA_E_INVALID, "need n_points > 0 and coordinates");
  std::vector<real> h;
  TRY(from_device(c, xyz, 3 * n, h, "landmark coordinates"));
  return SQRTBA_API(set_landmarks)(c, n, h.data());
}

int32_t SQRTBA_API(set_observations_device)(sqrtba_ctx* c, int64_t n, const int32_t* cam, const int32_t* pt,
                                            const real* uv) {
  if (!c) return SQRTBA_E_INVALID;
  if (n <= 0) return fail(c, SQRTBA_E_INVALID, "need n_obs > 0 and observation arrays");
  std::vector<int32_t> hc, hp;
  std::vector<real> huv;
  TRY(from_device(c, cam, n, hc, "observation cameras"));
  TRY(from_device(c, pt, n, hp, "observation landmarks"));
  TRY(from_device(c, uv, 2 * n, huv, "observation pixels"));
  return SQRTBA_API(set_observations)(c, n, hc.data(), hp.data(), huv.data());
}

int32_t SQRTBA_API(get_cameras_device)(sqrtba_ctx* c, real* params) {
  if (!c) return SQRTBA_E_INVALID;
  if (c->h.NC < 0) return fail(c, SQRTBA_E_STATE, "no cameras");
  std::vector<real> h(9 * (size_t)c->h.NC);
  TRY(SQRTBA_API(get_cameras)(c, h.data()));
  return to_device(c, params, h, "camera output");
}

int32_t SQRTBA_API(get_landmarks_device)(sqrtba_ctx* c, real* xyz) {
  if (!c) return SQRTBA_E_INVALID;
  if (c->h.NL < 0) return fail(c, SQRTBA_E_STATE, "no landmarks");
  std::vector<real> h(3 * (size_t)c->h.NL);
  TRY(SQRTBA_API(get_landmarks)(c, h.data()));
  return to_device(c, xyz, h, "landmark output");
}

int32_t SQRTBA_API(debug_bookkeeping)(const sqrtba_ctx* c, int64_t* n_active, int64_t* obs_perm, int64_t* lm_off,
                                 uint8_t* lm_active, uint8_t* cam_active) {
  if (!c || !n_active) return SQRTBA_E_INVALID;
  if (!c->h.obs_set) return SQRTBA_E_STATE;
  const HostData& h = c->h;
  *n_active = h.NO;
  if (obs_perm) std::memcpy(obs_perm, h.obs_perm.data(), 8 * h.NO);
  if (lm_off) std::memcpy(lm_off, h.lm_off.data(), 8 * (h.NL + 1));
  if (lm_active) std::memcpy(lm_active, h.lm_active.data(), h.NL);
  if (cam_active) std::memcpy(cam_active, h.cam_active.data(), h.NC);
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_linearization)(sqrtba_ctx* c, real* r, real* Jp, real* Jl) {
  if (!c) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  const int64_t NO = c->h.NO;
  real* buf = nullptr;
  HIP_TRY(c, hipMalloc(&buf, sizeof(real) * 26 * (NO > 0 ? NO : 1)));
  hipError_t e = launch_debug_linearization(c->d, c->L, buf, buf + 2 * NO, buf + 20 * NO);
  std::vector<real> hbuf(26 * NO);
  if (e == hipSuccess) e = hipMemcpyAsync(hbuf.data(), buf, hbuf.size() * sizeof(real), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(c, SQRTBA_E_HIP, "debug_linearization: %s", hipGetErrorString(e));
  if (r) std::memcpy(r, hbuf.data(), sizeof(real) * 2 * NO);
  if (Jp) std::memcpy(Jp, hbuf.data() + 2 * NO, sizeof(real) * 18 * NO);
  if (Jl) std::memcpy(Jl, hbuf.data() + 20 * NO, sizeof(real) * 6 * NO);
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_scales)(sqrtba_ctx* c, real* s_cam, real* s_pt) {
  if (!c) return SQRTBA_E_INVALID;
  if (!c->marginalized) return fail(c, SQRTBA_E_STATE, "scales need linearize and marginalize");
  const HostData& h = c->h;
  if (s_cam) {
    HIP_TRY(c, hipMemcpyAsync(s_cam, c->d.s_cam, sizeof(real) * 9 * h.NC, hipMemcpyDeviceToHost, c->stream));
  }
  std::vector<real> lmd(LMD_STRIDE * h.NS);
  if (h.NS) HIP_TRY(c, hipMemcpyAsync(lmd.data(), c->d.lmd, sizeof(real) * lmd.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (s_pt)
    for (int64_t l = 0; l < h.NL; ++l)
      for (int j = 0; j < 3; ++j)
        s_pt[3 * l + j] = h.lm_slot[l] >= 0 ? lmd[LMD_STRIDE * h.lm_slot[l] + LMD_SL + j] : 1.0f;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_rcs_matvec)(sqrtba_ctx* c, int32_t m, const real* v, real* out) {
  if (!c || m < 0 || (m > 0 && (!v || !out))) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "rcs_matvec needs damp");
  const int64_t N = 9 * c->h.NC;
  real* buf = nullptr;
  HIP_TRY(c, hipMalloc(&buf, sizeof(real) * 2 * N));
  hipError_t e = hipSuccess;
  for (int32_t i = 0; i < m && e == hipSuccess; ++i) {
    e = hipMemcpyAsync(buf, v + N * i, sizeof(real) * N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_matvec_only(c->d, c->L, buf, buf + N);
    if (e == hipSuccess) e = hipMemcpyAsync(out + N * i, buf + N, sizeof(real) * N, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(c, SQRTBA_E_HIP, "rcs_matvec: %s", hipGetErrorString(e));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(rcs_matvec_noalloc)(sqrtba_ctx* c, const real* v, real* out) {
  if (!c || !v || !out) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "rcs_matvec_noalloc needs damp");
  if (c->opt.landmark_blocks != 0) return fail(c, SQRTBA_E_UNSUPPORTED, "rcs_matvec_noalloc: explicit landmark blocks only");
  const uint64_t need = sizeof(real) * (uint64_t)noalloc_elems(c->h.NC, c->h.z_floats, c->h.hz_floats);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(c, SQRTBA_E_UNSUPPORTED, "rcs_matvec_noalloc: the product needs %llu bytes of scratch, the limit is %llu",
                (unsigned long long)need, (unsigned long long)NOALLOC_SCRATCH_BYTES);
  LAUNCH(c, launch_matvec_noalloc(c->d, c->L, c->noalloc_scratch, c->h.z_floats, v, out));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_rhs)(sqrtba_ctx* c, real* rhs) {
  if (!c || !rhs) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "rhs needs damp");
  LAUNCH(c, launch_precond_rhs(c->d, c->L));
  HIP_TRY(c, hipMemcpyAsync(rhs, c->d.vb, sizeof(real) * 9 * c->h.NC, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_precond)(sqrtba_ctx* c, real* minv) {
  if (!c || !minv) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "precond needs damp");
  LAUNCH(c, launch_precond_rhs(c->d, c->L));
  HIP_TRY(c, hipMemcpyAsync(minv, c->d.minv, sizeof(real) * 81 * c->h.NC, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_block)(sqrtba_ctx* c, int64_t pt, int32_t* k_out, real* out, real* factors) {
  if (!c || !k_out) return SQRTBA_E_INVALID;
  if (!c->marginalized) return fail(c, SQRTBA_E_STATE, "block needs marginalize");
  const HostData& h = c->h;
  if (pt < 0 || pt >= h.NL) return fail(c, SQRTBA_E_INVALID, "landmark out of range");
  const int32_t s = h.lm_slot[pt];
  if (s < 0) {
    *k_out = 0;
    return SQRTBA_OK;
  }
  const int64_t k = h.slot_k[s], W = width_of_h(k), C = 9 * k + 4;
  *k_out = (int32_t)k;
  if (!out && !factors) return SQRTBA_OK;
  if (c->opt.landmark_blocks != 0) {
    if (out) return fail(c, SQRTBA_E_UNSUPPORTED, "only explicit landmark blocks store block rows");
    std::vector<real> lmd(LMD_STRIDE);
    HIP_TRY(c, hipMemcpyAsync(lmd.data(), c->d.lmd + LMD_STRIDE * s, sizeof(real) * LMD_STRIDE, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::memcpy(factors, lmd.data(), sizeof(real) * 24);
    return SQRTBA_OK;
  }
  std::vector<real> T(3 * W), B(2 * k * W), rho(2 * k), lmd(LMD_STRIDE);
  HIP_TRY(c, hipMemcpyAsync(T.data(), c->d.poolT + h.slot_toff[s], sizeof(real) * T.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(B.data(), c->d.poolB + h.slot_boff[s], sizeof(real) * B.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(rho.data(), c->d.rhoB + 2 * h.slot_obs0[s], sizeof(real) * rho.size(), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(lmd.data(), c->d.lmd + LMD_STRIDE * s, sizeof(real) * LMD_STRIDE, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (out) {
    std::fill(out, out + (2 * k + 3) * C, 0.f);
    const real* R = lmd.data() + LMD_R;
    const real Rfull[9] = {R[0], R[1], R[2], 0, R[3], R[4], 0, 0, R[5]};
    for (int i = 0; i < 3; ++i) {
      for (int64_t j = 0; j < 9 * k; ++j) out[i * C + j] = T[i * W + j];
      for (int j = 0; j < 3; ++j) out[i * C + 9 * k + j] = Rfull[3 * i + j];
      out[i * C + 9 * k + 3] = lmd[LMD_QR + i];
    }
    for (int64_t i = 0; i < 2 * k; ++i) {
      for (int64_t j = 0; j < 9 * k; ++j) out[(3 + i) * C + j] = B[i * W + j];
      out[(3 + i) * C + 9 * k + 3] = rho[i];
    }
  }
  if (factors) std::memcpy(factors, lmd.data(), sizeof(real) * 24);
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_solution)(sqrtba_ctx* c, real* dxp, real* dxl) {
  if (!c) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  if (dxp) HIP_TRY(c, hipMemcpyAsync(dxp, c->d.vx, sizeof(real) * 9 * c->h.NC, hipMemcpyDeviceToHost, c->stream));
  if (dxl) HIP_TRY(c, hipMemcpyAsync(dxl, c->d.dxl, sizeof(real) * 3 * c->h.NL, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_set_pose_increment)(sqrtba_ctx* c, const real* dxp) {
  if (!c || !dxp) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "set_pose_increment needs damp");
  HIP_TRY(c, hipMemcpyAsync(c->d.vx, dxp, sizeof(real) * 9 * c->h.NC, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->solved = true;
  c->backsubbed = c->updated = false;
  return SQRTBA_OK;
}

#ifndef SQRTBA_FP64  // the learned preconditioner and its training are FP32 only

int32_t SQRTBA_API(mlp_num_params)(void) { return MLP_PARAMS; }

int32_t SQRTBA_API(mlp_init)(sqrtba_ctx* c, uint64_t seed) {
  if (!c) return SQRTBA_E_INVALID;
  return init_params(c, seed);
}

int32_t SQRTBA_API(mlp_set_params)(sqrtba_ctx* c, const float* params) {
  if (!c || !params) return SQRTBA_E_INVALID;
  for (int i = 0; i < MLP_PARAMS; ++i)
    if (!std::isfinite(params[i])) return fail(c, SQRTBA_E_NONFINITE, "parameter %d is not finite", i);
  TRY(ensure_learned(c));
  HIP_TRY(c, hipMemcpyAsync(c->ln.w32, params, 4 * (size_t)MLP_PARAMS, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ln.adam_m, 0, 4 * (size_t)MLP_PARAMS, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ln.adam_v, 0, 4 * (size_t)MLP_PARAMS, c->stream));
  LAUNCH(c, launch_to_bf16(learn_dev(c), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->ln.adam_step = 0;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(mlp_get_params)(sqrtba_ctx* c, float* params) {
  if (!c || !params) return SQRTBA_E_INVALID;
  if (!c->ln.alloc) return fail(c, SQRTBA_E_STATE, "no network: call sqrtba_mlp_init or sqrtba_mlp_set_params");
  HIP_TRY(c, hipMemcpyAsync(params, c->ln.w32, 4 * (size_t)MLP_PARAMS, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(set_preconditioner)(sqrtba_ctx* c, int32_t mode) {
  if (!c || (mode != 0 && mode != 1)) return SQRTBA_E_INVALID;
  if (mode == 1 && !c->ln.alloc) return fail(c, SQRTBA_E_STATE, "no network: call sqrtba_mlp_init or sqrtba_mlp_set_params");
  c->ln.mode = mode;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(pcg_trace)(sqrtba_ctx* c, int32_t max_solves, int32_t iters_per_solve) {
  if (!c || max_solves < 0 || iters_per_solve < 0) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  auto& L = c->ln;
  for (void** p : {(void**)&L.t_feat, (void**)&L.t_lfac, (void**)&L.t_p, (void**)&L.t_q})
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  L.max_solves = L.iters_per_solve = L.n_solves = L.n_records = 0;
  L.h_rec_solve.clear();
  if (max_solves == 0 || iters_per_solve == 0) return SQRTBA_OK;
  const size_t NC = c->h.NC, recs = (size_t)max_solves * iters_per_solve;
  HIP_TRY(c, hipMalloc(&L.t_feat, 4 * 64 * NC * max_solves));
  HIP_TRY(c, hipMalloc(&L.t_lfac, 4 * 45 * NC * max_solves));
  HIP_TRY(c, hipMalloc(&L.t_p, 4 * 9 * NC * recs));
  HIP_TRY(c, hipMalloc(&L.t_q, 4 * 9 * NC * recs));
  L.max_solves = max_solves;
  L.iters_per_solve = iters_per_solve;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(trace_size)(const sqrtba_ctx* c, int32_t* n_solves, int32_t* n_records) {
  if (!c) return SQRTBA_E_INVALID;
  if (n_solves) *n_solves = c->ln.n_solves;
  if (n_records) *n_records = c->ln.n_records;
  return SQRTBA_OK;
}

static int grow_training(sqrtba_ctx* c, int n) {
  auto& L = c->ln;
  const int tiles = mlp_tiles(n);
  if (tiles > L.part_tiles) {
    if (L.part) (void)hipFree(L.part);
    if (L.loss_part) (void)hipFree(L.loss_part);
    L.part = nullptr;
    L.loss_part = nullptr;
    HIP_TRY(c, hipMalloc(&L.part, 4 * (size_t)MLP_PARAMS * tiles));
    HIP_TRY(c, hipMalloc(&L.loss_part, 8 * (size_t)tiles));
    L.part_tiles = tiles;
  }
  if (n > L.s_cap) {
    if (L.s_rec) (void)hipFree(L.s_rec);
    if (L.s_cam) (void)hipFree(L.s_cam);
    L.s_rec = L.s_cam = nullptr;
    HIP_TRY(c, hipMalloc(&L.s_rec, 4 * (size_t)n));
    HIP_TRY(c, hipMalloc(&L.s_cam, 4 * (size_t)n));
    L.s_cap = n;
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(mlp_train)(sqrtba_ctx* c, int32_t steps, int32_t batch, double lr, uint64_t seed, double* losses) {
  if (!c || steps < 0 || batch <= 0 || !(lr >= 0)) return SQRTBA_E_INVALID;
  auto& L = c->ln;
  if (!L.alloc) return fail(c, SQRTBA_E_STATE, "no network: call sqrtba_mlp_init or sqrtba_mlp_set_params");
  if (L.n_records == 0) return fail(c, SQRTBA_E_STATE, "no traced PCG iterations: enable sqrtba_pcg_trace and solve");
  TRY(grow_training(c, batch));
  if (L.rec_solve) (void)hipFree(L.rec_solve);
  L.rec_solve = nullptr;
  HIP_TRY(c, hipMalloc(&L.rec_solve, 4 * (size_t)L.n_records));
  HIP_TRY(c, hipMemcpyAsync(L.rec_solve, L.h_rec_solve.data(), 4 * (size_t)L.n_records, hipMemcpyHostToDevice, c->stream));
  std::vector<int32_t> cams;
  for (int64_t q = 0; q < c->h.NC; ++q)
    if (c->h.cam_active[q]) cams.push_back((int32_t)q);
  if (cams.empty()) return fail(c, SQRTBA_E_STATE, "no active camera");
  std::mt19937_64 rng(seed);
  std::uniform_int_distribution<int32_t> ur(0, L.n_records - 1), uc(0, (int32_t)cams.size() - 1);
  std::vector<int32_t> hr(batch), hc(batch);
  const int tiles = mlp_tiles(batch);
  std::vector<double> lp(tiles);
  SampleSrc src{};
  src.mode = 1;
  src.NC = (int)c->h.NC;
  src.rec = L.s_rec;
  src.cam = L.s_cam;
  src.rec_solve = L.rec_solve;
  src.t_feat = L.t_feat;
  src.t_lfac = L.t_lfac;
  src.t_p = L.t_p;
  src.t_q = L.t_q;
  for (int st = 0; st < steps; ++st) {
    for (int i = 0; i < batch; ++i) {
      hr[i] = ur(rng);
      hc[i] = cams[uc(rng)];
    }
    HIP_TRY(c, hipMemcpyAsync(L.s_rec, hr.data(), 4 * (size_t)batch, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(L.s_cam, hc.data(), 4 * (size_t)batch, hipMemcpyHostToDevice, c->stream));
    LAUNCH(c, launch_mlp_grad(learn_dev(c), src, batch, L.part, L.loss_part, L.grad, c->stream));
    if (lr > 0) LAUNCH(c, launch_adam(learn_dev(c), L.grad, (float)lr, ++L.adam_step, c->stream));
    HIP_TRY(c, hipMemcpyAsync(lp.data(), L.loss_part, 8 * (size_t)tiles, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0;
    for (double v : lp) tot += v;
    if (losses) losses[st] = tot / batch;
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(mlp_eval)(sqrtba_ctx* c, int32_t n, const float* feats, const float* lfac, const float* p,
                        const float* q, double* loss, float* grad) {
  if (!c || n <= 0 || !feats || !lfac || !p || !q) return SQRTBA_E_INVALID;
  auto& L = c->ln;
  if (!L.alloc) return fail(c, SQRTBA_E_STATE, "no network: call sqrtba_mlp_init or sqrtba_mlp_set_params");
  TRY(grow_training(c, n));
  float* buf = nullptr;
  HIP_TRY(c, hipMalloc(&buf, 4 * (size_t)n * (64 + 45 + 18)));
  SampleSrc src{};
  src.mode = 0;
  src.a_feat = buf;
  src.a_lfac = buf + 64 * (size_t)n;
  src.a_p = buf + 109 * (size_t)n;
  src.a_q = buf + 118 * (size_t)n;
  hipError_t e = hipMemcpyAsync(buf, feats, 4 * 64 * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(buf + 64 * (size_t)n, lfac, 4 * 45 * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(buf + 109 * (size_t)n, p, 4 * 9 * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(buf + 118 * (size_t)n, q, 4 * 9 * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_mlp_grad(learn_dev(c), src, n, L.part, L.loss_part, L.grad, c->stream);
  const int tiles = mlp_tiles(n);
  std::vector<double> lp(tiles);
  if (e == hipSuccess) e = hipMemcpyAsync(lp.data(), L.loss_part, 8 * (size_t)tiles, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && grad) e = hipMemcpyAsync(grad, L.grad, 4 * (size_t)MLP_PARAMS, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(c, SQRTBA_E_HIP, "mlp_eval: %s", hipGetErrorString(e));
  if (loss) {
    double tot = 0;
    for (double v : lp) tot += v;
    *loss = tot / n;
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(learned_stats)(const sqrtba_ctx* c, int64_t* learned_solves, int64_t* fallbacks, int64_t* wasted_iters) {
  if (!c) return SQRTBA_E_INVALID;
  if (learned_solves) *learned_solves = c->ln.learned_solves;
  if (fallbacks) *fallbacks = c->ln.fallbacks;
  if (wasted_iters) *wasted_iters = c->ln.wasted_iters;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_features)(sqrtba_ctx* c, float* feats, float* lfac) {
  if (!c) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "features need damp");
  LAUNCH(c, launch_precond_rhs(c->d, c->L));
  if (feats) HIP_TRY(c, hipMemcpyAsync(feats, c->d.feats, 4 * 64 * (size_t)c->h.NC, hipMemcpyDeviceToHost, c->stream));
  if (lfac) HIP_TRY(c, hipMemcpyAsync(lfac, c->d.lfac, 4 * 45 * (size_t)c->h.NC, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(debug_learned_precond)(sqrtba_ctx* c, float* minv) {
  if (!c || !minv) return SQRTBA_E_INVALID;
  if (!c->damped) return fail(c, SQRTBA_E_STATE, "needs damp");
  if (!c->ln.alloc) return fail(c, SQRTBA_E_STATE, "no network");
  LAUNCH(c, launch_precond_rhs(c->d, c->L));
  LAUNCH(c, launch_mlp_precond(c->d, learn_dev(c), c->stream));
  HIP_TRY(c, hipMemcpyAsync(minv, c->d.minv, 4 * 81 * (size_t)c->h.NC, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

#endif  // SQRTBA_FP64

int32_t SQRTBA_API(profile_enable)(sqrtba_ctx* c, int32_t on) {
  if (!c) return SQRTBA_E_INVALID;
  if (c->stream) HIP_TRY(c, hipStreamSynchronize(c->stream));
  flush_profile(c);
  c->prof = sqrtba_profile{};
  c->prof_on = on != 0;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(profile_get)(const sqrtba_ctx* c, sqrtba_profile* out) {
  if (!c || !out) return SQRTBA_E_INVALID;
  *out = c->prof;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(save_state)(sqrtba_ctx* c) {
  if (!c) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  HIP_TRY(c, hipMemcpyAsync(c->d.cam_snap, c->d.cam, sizeof(real) * 16 * c->h.NC, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d.pts_snap, c->d.pts, sizeof(real) * 4 * c->h.NL, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->snapshot = true;
  return SQRTBA_OK;
}

int32_t SQRTBA_API(restore_state)(sqrtba_ctx* c) {
  if (!c) return SQRTBA_E_INVALID;
  if (!c->uploaded || !c->snapshot) return fail(c, SQRTBA_E_STATE, "restore_state needs save_state");
  HIP_TRY(c, hipMemcpyAsync(c->d.cam, c->d.cam_snap, sizeof(real) * 16 * c->h.NC, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d.pts, c->d.pts_snap, sizeof(real) * 4 * c->h.NL, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->linearized = c->marginalized = c->damped = c->solved = c->backsubbed = c->updated = false;
  return SQRTBA_OK;
}

}  // extern "C"

// ---- launch shapes and autotuner

namespace {

bool valid_tuning(const sqrtba_tuning& t) {
  const int r = t.huge_rows, e = t.rows_min_k, p = t.persist_wgs;
  return (r == 64 || r == 128 || r == 256 || r == 512 || r == 1024) && (e == 114 || e == 61 || e == 29) &&
         (t.huge_side == 0 || t.huge_side == 1) && (t.large_separate == 0 || t.large_separate == 1) &&
         (t.small_rows == 4 || t.small_rows == 8) && (p == 0 || p == 1024 || p == 2048 || p == 4096) &&
         (t.stream_loads >= 0 && t.stream_loads <= 3);
}

sqrtba_tuning current_tuning(const sqrtba_ctx* c) {
  sqrtba_tuning t;
  t.rows_min_k = c->L.rows_min_k;
  t.huge_rows = c->L.huge_rows;
  t.huge_side = c->L.huge_side;
  t.large_separate = c->L.large_sep;
  t.small_rows = c->L.mv_rbs ? 8 : 4;
  t.persist_wgs = c->L.persist;
  t.stream_loads = c->L.nt;
  return t;
}

int apply_tuning(sqrtba_ctx* c, const sqrtba_tuning& t) {
  TRY(set_row_blocks(c, t.rows_min_k, t.huge_rows));
  c->L.huge_side = t.huge_side;
  c->L.large_sep = t.large_separate;
  c->L.mv_rbs = t.small_rows == 8 ? 1 : 0;
  c->L.persist = t.persist_wgs;
  c->L.nt = t.stream_loads;
  if (c->graph) {  // the captured PCG iterations hold the old launches
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  return SQRTBA_OK;
}

// Mean milliseconds of one product over `reps` back-to-back launches (after two
// untimed ones), HIP events on the context stream.
// Average duration of one product over `reps` back-to-back products, launched as
// one captured HIP graph as the PCG iterations are (graph-launched products have
// no launch gaps between their kernels and their side-stream branch); HIP events
// around the second launch of the graph.
int time_products(sqrtba_ctx* c, int reps, double* ms) {
  hipEvent_t e0 = take_event(c), e1 = take_event(c);
  if (!e0 || !e1) return fail(c, SQRTBA_E_HIP, "no events");
  c->event_pool.push_back(e0);
  c->event_pool.push_back(e1);
  LAUNCH(c, launch_prescale_z(c->d, c->L));
  hipGraph_t g = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < reps && le == hipSuccess; ++i) le = launch_matvec_timing(c->d, c->L);
  const hipError_t ee = hipStreamEndCapture(c->stream, &g);
  if (le != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(c, SQRTBA_E_HIP, "product capture: %s", hipGetErrorString(le != hipSuccess ? le : ee));
  }
  hipGraphExec_t ge = nullptr;
  hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(c, SQRTBA_E_HIP, "product graph instantiate: %s", hipGetErrorString(e));
  e = hipGraphLaunch(ge, c->stream);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  if (e == hipSuccess) e = hipGraphLaunch(ge, c->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
  (void)hipGraphExecDestroy(ge);
  if (e != hipSuccess) return fail(c, SQRTBA_E_HIP, "product timing: %s", hipGetErrorString(e));
  *ms = (double)f / reps;
  return SQRTBA_OK;
}

}  // namespace

int32_t SQRTBA_API(time_product)(sqrtba_ctx* c, int32_t reps, double* ms, double* bytes) {
  if (!c || reps <= 0 || !ms) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  TRY(time_products(c, reps, ms));
  if (bytes) {
    double b = 0.0;
    for (int p = 0; p < c->h.P; ++p)
      if (c->active[p]) b += c->mv_bytes[p];
    *bytes = b;
  }
  return SQRTBA_OK;
}

int32_t SQRTBA_API(get_tuning)(sqrtba_ctx* c, sqrtba_tuning* out) {
  if (!c || !out) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  *out = current_tuning(c);
  return SQRTBA_OK;
}

int32_t SQRTBA_API(set_tuning)(sqrtba_ctx* c, const sqrtba_tuning* t) {
  if (!c || !t || !valid_tuning(*t)) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  TRY(apply_tuning(c, *t));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return SQRTBA_OK;
}

int32_t SQRTBA_API(autotune)(sqrtba_ctx* c, int32_t reps, sqrtba_tuning* best, sqrtba_tuning_trial* trials,
                        int32_t max_trials, int32_t* n_trials) {
  if (!c || max_trials < 0) return SQRTBA_E_INVALID;
  TRY(ensure_uploaded(c));
  if (reps <= 0) reps = 10;
  std::vector<sqrtba_tuning_trial> tr;
  auto measure = [&](const sqrtba_tuning& t, double* ms) -> int {
    TRY(apply_tuning(c, t));
    TRY(time_products(c, reps, ms));
    tr.push_back({t, *ms});
    return SQRTBA_OK;
  };
  sqrtba_tuning cur = current_tuning(c);
  double cur_ms = 0.0;
  TRY(measure(cur, &cur_ms));
  // a candidate replaces the current shape when it is faster by more than `margin`
  auto try_field = [&](int sqrtba_tuning::*field, std::initializer_list<int> values, double margin = 0.0) -> int {
    for (int v : values) {
      if (cur.*field == v) continue;
      sqrtba_tuning t = cur;
      t.*field = v;
      double ms = 0.0;
      TRY(measure(t, &ms));
      if (ms < (1.0 - margin) * cur_ms) {
        cur = t;
        cur_ms = ms;
      }
    }
    return SQRTBA_OK;
  };
  // bucket edge first (it decides which kernels run), then the shapes of the
  // kernels that do run
  // (the shapes are those of the explicit-block product kernels; with implicit
  // blocks only the current shape is timed)
  if (!c->d.implicit) {
    if (c->L.n45 > 0) TRY(try_field(&sqrtba_tuning::rows_min_k, {114, 61, 29}));
    if (c->L.rows_n > 0) {
      TRY(try_field(&sqrtba_tuning::huge_rows, {64, 128, 256, 1024}));
      TRY(try_field(&sqrtba_tuning::huge_side, {0, 1}));
    }
    if (c->L.n45 > c->L.rows_n) TRY(try_field(&sqrtba_tuning::large_separate, {0, 1}));
    TRY(try_field(&sqrtba_tuning::small_rows, {4, 8}));
    TRY(try_field(&sqrtba_tuning::persist_wgs, {0, 1024, 2048, 4096}));
    // non-temporal loads only on a clear gain: a solve also rereads the blocks
    // outside the product (back-substitution), which they may slow
    if (c->L.n45 > 0)
      TRY(try_field(&sqrtba_tuning::stream_loads, {0, 1, 2, 3}, 0.01));
    else
      TRY(try_field(&sqrtba_tuning::stream_loads, {0, 2}, 0.01));
  }
  TRY(apply_tuning(c, cur));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (best) *best = cur;
  if (trials)
    for (int i = 0; i < (int)tr.size() && i < max_trials; ++i) trials[i] = tr[i];
  if (n_trials) *n_trials = (int32_t)tr.size();
  return SQRTBA_OK;
}
