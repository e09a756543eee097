// hers_api.cpp -- the C ABI of libhers (include/hers.h): context set-up,
// size queries, argument checks and the launch sequences of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/hers.h"
#include "internal.h"
#include "kernels.h"
#include "params.h"

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

void hers::set_last_error(const std::string& msg) { g_err = msg; }

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(HERS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// "mac_variant" of the multiply-accumulate with the inverse NTT of the
// accumulators fused in (k_mac_intt, n <= 4096); 0 .. 11 are k_mac schedules
#define MAC_FUSED_INTT 12

struct hers_ctx {
  int num_cus = 256;
  hers_params prm;
  hers::HostTables host;
  int device;
  std::vector<void*> allocs;
  DevTabs T;
  bool keys_loaded;
  int mac_variant = 8;   // k_mac schedule (see hers_set_option)
  // overlapped search: chunk count (0 automatic, 1 off), the stream the
  // per-block epilogue runs on, and its events (MAC done, join, one per
  // workspace region)
  int overlap_chunks = 0;
  int dec_fused = 1;                // decryption and decoding in one kernel where it fits
  int mac_wgs_per_cu = 0;   // multiply-accumulate grid, workgroups per CU (0 = 8)
  int64_t relin_fuse_min_wgs = 0;   // fused relinearization from this many workgroups (0 = 8 per CU)
  int mb_variant = 0;               // multi-probe multiply-accumulate schedule (launch_mac_multi)
  int mb_group = MB_PROBES;         // probes per group of the batched search
  // rotation keys of the re-rank stage, NTT form [steps][L][2][k][n]
  uint64_t* rk_ntt = nullptr;
  uint64_t* rk_ntt_sh = nullptr;
  int rk_steps = 0;
  // secret key in NTT form for decryptions without a key argument
  uint64_t* sk_ntt = nullptr;
  bool sk_loaded = false;
  // input checks: a device flag word and its pinned host copy
  uint32_t* flag_dev = nullptr;
  uint32_t* flag_host = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t ev_mac = nullptr, ev_join = nullptr;
  std::vector<hipEvent_t> ev_free;
  // per-stage timing
  struct Rec { std::string stage; hipEvent_t a, b; };
  bool prof_on = false;
  std::vector<std::string> prof_sel;   // stages timed while profiling is on (empty: all)
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::string, std::pair<double, uint64_t>> totals;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <class T>
int upload(hers_ctx* c, const std::vector<T>& v, const T** dst) {
  void* p = nullptr;
  if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) return fail(HERS_ENOMEM, "hipMalloc of library tables failed");
  c->allocs.push_back(p);
  HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = (const T*)p;
  return HERS_OK;
}

int alloc_dev(hers_ctx* c, size_t bytes, void** dst) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(HERS_ENOMEM, "hipMalloc of library tables failed");
  c->allocs.push_back(p);
  *dst = p;
  return HERS_OK;
}

hipEvent_t take_event(hers_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events on its stream while profiling is enabled.
static bool selected(const hers_ctx* c, const char* stage) {
  if (c->prof_sel.empty()) return true;
  for (const auto& s : c->prof_sel)
    if (s == stage) return true;
  return false;
}

struct StageTimer {
  hers_ctx* c;
  hipStream_t s;
  hipEvent_t a = nullptr;
  const char* stage;
  StageTimer(hers_ctx* ctx, const char* name, hipStream_t stream) : c(ctx), s(stream), stage(name) {
    if (c->prof_on && selected(c, name) && (a = take_event(c))) (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) { c->pool.push_back(a); return; }
    (void)hipEventRecord(b, s);
    c->pending.push_back({stage, a, b});
  }
};

#define TIMED(ctx, name, stream, expr) \
  do {                                 \
    StageTimer st_(ctx, name, stream); \
    HIP_TRY(expr);                     \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// per-block workspace of the search: accumulators u32 [3][K][n] + digits u64 [L][k][n]
size_t search_ws_per_block(const HersConsts& C) {
  return align256((size_t)3 * C.K * C.n * 4) + align256((size_t)C.L * C.k * C.n * 8);
}

size_t decrypt_ws_fixed(const HersConsts& C) { return align256((size_t)2 * C.k * C.n * 8); }
size_t decrypt_ws_per_block(const HersConsts& C) { return align256((size_t)C.k * C.n * 8); }

size_t enc_ws_per_block(const HersConsts& C, int32_t d, bool canon_given) {
  size_t b = align256((size_t)d * C.n * 4);
  if (!canon_given) b += align256((size_t)d * 2 * C.k * C.n * 8);
  return b;
}

// re-rank workspace per ciphertext: gathered search form, accumulators,
// digits, one ping-pong ciphertext
size_t rerank_ws_per_ct(const HersConsts& C) {
  return align256((size_t)C.K * 2 * C.n * 4) + search_ws_per_block(C) + align256((size_t)2 * C.k * C.n * 8);
}

int check_d(const hers_ctx* c, int32_t d) {
  if (d < 1 || (uint32_t)d > c->prm.d_max) return fail(HERS_EDIM, "d must be in [1, d_max]");
  return HERS_OK;
}

// Search-form buffer lengths against (m, d): the probe must be the search form
// of exactly d dimensions, the gallery whole blocks of d dimensions covering
// the m items (a probe or gallery made for another d is a mismatch).
int check_search_buffers(const hers_ctx* c, int64_t m, int32_t d, uint64_t gallery_words, uint64_t probe_words) {
  const HersConsts& C = c->host.C;
  const uint64_t blk = (uint64_t)C.K * d * 2 * C.n;
  if (probe_words != blk) return fail(HERS_EDIM, "probe buffer length is not the search form of d dimensions");
  if (gallery_words % blk || gallery_words / blk < (uint64_t)((m + C.n - 1) / C.n))
    return fail(HERS_EDIM, "gallery buffer length is not whole blocks of d dimensions covering the m items");
  return HERS_OK;
}

// Runs a checking kernel that may set the context's flag word, reads the flag
// back and fails with `code` if it was set.  Synchronises the stream.
template <class F>
int flag_check(hers_ctx* c, hipStream_t s, F&& launch, int code, const char* msg) {
  HIP_TRY(hipMemsetAsync(c->flag_dev, 0, sizeof(uint32_t), s));
  HIP_TRY(launch());
  HIP_TRY(hipMemcpyAsync(c->flag_host, c->flag_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (*c->flag_host) return fail(code, msg);
  return HERS_OK;
}

// Values of a [rows][ld] int32 device array (columns 0 .. cols - 1) must lie
// in [-feature_bound, feature_bound] (Sec. 3.2, "Encoding Scheme": every
// score then stays below t / 2 and is recovered exactly).
int check_features(hers_ctx* c, const int32_t* v, int64_t ld, int32_t rows, int64_t cols, hipStream_t s) {
  return flag_check(c, s, [&] {
    return hers::launch_check_features(v, ld, rows, cols, (int32_t)c->prm.feature_bound, c->flag_dev,
                                       (uint32_t)c->num_cus, s);
  }, HERS_ERANGE, "a feature or query value lies outside [-feature_bound, feature_bound]");
}

}  // namespace

extern "C" {

const char* hers_last_error(void) { return g_err.c_str(); }

int hers_params_resolve(const hers_params* params, hers_info* out) {
  if (!params || !out) return fail(HERS_EINVAL, "null argument");
  std::string e = hers::resolve(*params, out);
  if (!e.empty()) return fail(HERS_EPARAM, e);
  return HERS_OK;
}

static std::vector<double> to_double(const std::vector<uint64_t>& v) { return std::vector<double>(v.begin(), v.end()); }

static std::vector<double> qf_consts(const HersConsts& C) {
  std::vector<double> f(3 * HC_MAXQ, 0.0);
  for (uint32_t i = 0; i < C.k; ++i) {
    f[i] = (double)C.q[i];
    f[HC_MAXQ + i] = 1.0 / (double)C.q[i];
    f[2 * HC_MAXQ + i] = (double)C.q_ninv[i];
  }
  return f;
}

int hers_ctx_create(const hers_params* params, int device, hers_ctx** out) {
  if (!params || !out) return fail(HERS_EINVAL, "null argument");
  *out = nullptr;
  hers_ctx* c = new hers_ctx();
  c->prm = *params;
  c->device = device;
  c->keys_loaded = false;
  std::string e = hers::precompute(*params, &c->host);
  if (!e.empty()) { delete c; return fail(HERS_EPARAM, e); }
  DeviceGuard g(device);
  int rc = HERS_OK;
  const HersConsts& C = c->host.C;
  std::vector<HersConsts> cv(1, C);
  const HersConsts* dC = nullptr;
  void *pk = nullptr, *pks = nullptr, *rl = nullptr, *rls = nullptr;
  if ((rc = upload(c, cv, &dC)) ||
      (rc = upload(c, c->host.qtw, &c->T.qtw)) || (rc = upload(c, c->host.qtw_sh, &c->T.qtw_sh)) ||
      (rc = upload(c, c->host.qitw, &c->T.qitw)) || (rc = upload(c, c->host.qitw_sh, &c->T.qitw_sh)) ||
      (rc = upload(c, c->host.ptw, &c->T.ptw)) || (rc = upload(c, c->host.ptw_sh, &c->T.ptw_sh)) ||
      (rc = upload(c, c->host.pitw, &c->T.pitw)) || (rc = upload(c, c->host.pitw_sh, &c->T.pitw_sh)) ||
      (rc = upload(c, c->host.ttw, &c->T.ttw)) || (rc = upload(c, c->host.ttw_sh, &c->T.ttw_sh)) ||
      (rc = upload(c, c->host.titw, &c->T.titw)) || (rc = upload(c, c->host.titw_sh, &c->T.titw_sh)) ||
      (rc = upload(c, to_double(c->host.qtw), &c->T.qtw_f)) ||
      (rc = upload(c, to_double(c->host.qitw), &c->T.qitw_f)) ||
      (rc = upload(c, qf_consts(C), &c->T.qf)) ||
      (rc = alloc_dev(c, (size_t)2 * C.k * C.n * 8, &pk)) || (rc = alloc_dev(c, (size_t)2 * C.k * C.n * 8, &pks)) ||
      (rc = alloc_dev(c, (size_t)C.L * 2 * C.k * C.n * 8, &rl)) ||
      (rc = alloc_dev(c, (size_t)C.L * 2 * C.k * C.n * 8, &rls)) ||
      (rc = alloc_dev(c, 256, (void**)&c->flag_dev))) {
    std::string msg = g_err;
    hers_ctx_destroy(c);
    return fail(rc, msg);
  }
  if (hipHostMalloc((void**)&c->flag_host, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    c->flag_host = nullptr;
    hers_ctx_destroy(c);
    return fail(HERS_ENOMEM, "pinned host allocation failed");
  }
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_mac, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    hers_ctx_destroy(c);
    return fail(HERS_EDEVICE, "stream or event creation failed");
  }
  if (int rc2 = hers::scratch_setup(device)) {
    std::string msg = g_err;
    hers_ctx_destroy(c);
    return fail(rc2, msg);
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->num_cus = cus;
  c->T.C = dC;
  c->T.C_rare = dC;
  c->T.ntt_r = 4;
  c->T.rl_per = 8;
  c->T.nq = C.k;
  c->T.qf_ok = 1;
  for (uint32_t i = 0; i < C.k; ++i) c->T.qf_ok &= C.q[i] < (1ull << 45);
  c->T.pk_ntt = (uint64_t*)pk;
  c->T.pk_ntt_sh = (uint64_t*)pks;
  c->T.rlk_ntt = (uint64_t*)rl;
  c->T.rlk_ntt_sh = (uint64_t*)rls;
  *out = c;
  return HERS_OK;
}

void hers_ctx_destroy(hers_ctx* ctx) {
  if (!ctx) return;
  {
    DeviceGuard g(ctx->device);
    for (auto& r : ctx->pending) {
      (void)hipEventSynchronize(r.b);
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
    if (ctx->ev_mac) (void)hipEventDestroy(ctx->ev_mac);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->rk_ntt) (void)hipFree(ctx->rk_ntt);
    if (ctx->sk_ntt) (void)hipFree(ctx->sk_ntt);
    if (ctx->rk_ntt_sh) (void)hipFree(ctx->rk_ntt_sh);
    if (ctx->flag_host) (void)hipHostFree(ctx->flag_host);
    for (void* p : ctx->allocs) (void)hipFree(p);
  }
  delete ctx;
}

// Workspace of hers_topk: tile maxima, two ping-pong buffers of the generic
// passes, the k best tile maxima and the k * k filtered candidates.
struct TopkLayout {
  uint64_t tiles, nbest, maxes, pp, best, cand, total;
};

static TopkLayout topk_layout(uint64_t m, uint64_t k) {
  TopkLayout L{};
  L.tiles = (m + HERS_TOPK_TM - 1) >> HERS_TOPK_TM_LOG2;
  L.nbest = std::min<uint64_t>(k, L.tiles);
  const uint64_t first = std::max((L.tiles + HERS_TOPK_TILE - 1) / HERS_TOPK_TILE * L.nbest,
                                  (L.nbest * k + HERS_TOPK_TILE - 1) / HERS_TOPK_TILE * k);
  L.maxes = align256(L.tiles * 8);
  L.pp = align256(first * 8);
  L.best = align256(k * 8);
  L.cand = align256(L.nbest * k * 8);
  L.total = L.maxes + 2 * L.pp + L.best + L.cand;
  return L;
}

uint64_t hers_topk_workspace_bytes(int64_t m, int32_t k) {
  if (m < 1 || k < 1) return 0;
  if (k > HERS_TOPK_TILE_K) return hers::topk_large_state_bytes() + align256((uint64_t)k * 8);
  return topk_layout((uint64_t)m, (uint64_t)k).total;
}

// Top k of keys[0, count) by generic passes; the last pass (one workgroup)
// writes keys to out_keys, or decoded (index, score) when idx is set.
static int topk_reduce(hers_ctx* ctx, const uint64_t* keys, uint64_t count, uint32_t k, uint64_t* pp0, uint64_t* pp1,
                       uint64_t* out_keys, int64_t* idx, int32_t* val, hipStream_t s) {
  uint64_t* pp[2] = {pp0, pp1};
  int cur = 0;
  while (count > HERS_TOPK_TILE) {
    TIMED(ctx, "topk", s, hers::launch_topk_pass(nullptr, keys, count, k, pp[cur], nullptr, nullptr, s));
    keys = pp[cur];
    count = (count + HERS_TOPK_TILE - 1) / HERS_TOPK_TILE * k;
    cur ^= 1;
  }
  TIMED(ctx, "topk", s, hers::launch_topk_pass(nullptr, keys, count, k, out_keys, idx, val, s));
  return HERS_OK;
}

int hers_topk(hers_ctx* ctx, const int32_t* scores_dev, int64_t m, int32_t k, int64_t* idx_dev, int32_t* val_dev,
              void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || !scores_dev || !idx_dev || !val_dev) return fail(HERS_EINVAL, "null argument");
  if (m < 1 || m > ((int64_t)1 << 32)) return fail(HERS_EINVAL, "m must be in [1, 2^32]");
  if (k < 1 || k > HERS_TOPK_MAX_K || k > m) return fail(HERS_EINVAL, "k must be in [1, min(16384, m)]");
  if (!work_dev || work_bytes < hers_topk_workspace_bytes(m, k)) return fail(HERS_ESPACE, "workspace too small");
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  if (k > HERS_TOPK_TILE_K) {   // radix select, then ranks
    uint64_t* keys = (uint64_t*)((char*)work_dev + hers::topk_large_state_bytes());
    TIMED(ctx, "topk", s, hers::launch_topk_large(scores_dev, (uint64_t)m, (uint32_t)k, work_dev, keys, idx_dev,
                                                  val_dev, (uint32_t)ctx->num_cus, s));
    return HERS_OK;
  }
  if (m <= HERS_TOPK_TILE) {   // one tile: sort it directly
    TIMED(ctx, "topk", s, hers::launch_topk_pass(scores_dev, nullptr, (uint64_t)m, (uint32_t)k, nullptr, idx_dev,
                                                 val_dev, s));
    return HERS_OK;
  }
  const TopkLayout L = topk_layout((uint64_t)m, (uint64_t)k);
  char* w = (char*)work_dev;
  uint64_t* maxes = (uint64_t*)w;
  uint64_t* pp0 = (uint64_t*)(w + L.maxes);
  uint64_t* pp1 = (uint64_t*)(w + L.maxes + L.pp);
  uint64_t* best = (uint64_t*)(w + L.maxes + 2 * L.pp);
  uint64_t* cand = (uint64_t*)(w + L.maxes + 2 * L.pp + L.best);
  TIMED(ctx, "topk", s, hers::launch_topk_tilemax(scores_dev, (uint64_t)m, maxes, s));
  int rc = topk_reduce(ctx, maxes, L.tiles, (uint32_t)L.nbest, pp0, pp1, best, nullptr, nullptr, s);
  if (rc != HERS_OK) return rc;
  TIMED(ctx, "topk", s, hers::launch_topk_filter(scores_dev, (uint64_t)m, best, (uint32_t)L.nbest,
                                                 L.tiles >= (uint64_t)k, (uint32_t)k, cand, s));
  return topk_reduce(ctx, cand, L.nbest * (uint64_t)k, (uint32_t)k, pp0, pp1, nullptr, idx_dev, val_dev, s);
}

int hers_set_option(hers_ctx* ctx, const char* key, int64_t value) {
  if (!ctx || !key) return fail(HERS_EINVAL, "null argument");
  if (!std::strcmp(key, "mac_variant")) {
    const int64_t top = ctx->host.C.n <= 4096 ? MAC_FUSED_INTT : MAC_FUSED_INTT - 1;
    if (value < 0 || value > top) return fail(HERS_EINVAL, "mac_variant must be in [0, 11] (12 for n <= 4096)");
    ctx->mac_variant = (int)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "ntt_radix_log2")) {
    if (value < 1 || value > 4) return fail(HERS_EINVAL, "ntt_radix_log2 must be in [1, 4]");
    ctx->T.ntt_r = (uint32_t)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "dec_fused")) {
    if (value != 0 && value != 1) return fail(HERS_EINVAL, "dec_fused must be 0 or 1");
    ctx->dec_fused = (int)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "relin_lane_coeffs")) {
    if (value != 8 && value != 16) return fail(HERS_EINVAL, "relin_lane_coeffs must be 8 or 16");
    ctx->T.rl_per = (uint32_t)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "overlap_chunks")) {
    if (value < 0 || value > 256) return fail(HERS_EINVAL, "overlap_chunks must be in [0, 256]");
    ctx->overlap_chunks = (int)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "mac_wgs_per_cu")) {
    if (value < 0 || value > 64) return fail(HERS_EINVAL, "mac_wgs_per_cu must be in [0, 64]");
    ctx->mac_wgs_per_cu = (int)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "relin_fuse_min_wgs")) {
    if (value < 0 || value > (1ll << 30)) return fail(HERS_EINVAL, "relin_fuse_min_wgs must be in [0, 2^30]");
    ctx->relin_fuse_min_wgs = value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "mb_variant")) {
    if (value < 0 || value >= MB_VARIANTS) return fail(HERS_EINVAL, "mb_variant must be in [0, 4]");
    ctx->mb_variant = (int)value;
    return HERS_OK;
  }
  if (!std::strcmp(key, "mb_group")) {
    if (value < 1 || value > MB_PROBES) return fail(HERS_EINVAL, "mb_group must be in [1, 16]");
    ctx->mb_group = (int)value;
    return HERS_OK;
  }
  return fail(HERS_EINVAL, std::string("unknown option ") + key);
}

int hers_get_option(const hers_ctx* ctx, const char* key, int64_t* value) {
  if (!ctx || !key || !value) return fail(HERS_EINVAL, "null argument");
  if (!std::strcmp(key, "mac_variant")) {
    *value = ctx->mac_variant;
    return HERS_OK;
  }
  if (!std::strcmp(key, "ntt_radix_log2")) {
    *value = ctx->T.ntt_r;
    return HERS_OK;
  }
  if (!std::strcmp(key, "relin_lane_coeffs")) {
    *value = ctx->T.rl_per;
    return HERS_OK;
  }
  if (!std::strcmp(key, "dec_fused")) {
    *value = ctx->dec_fused;
    return HERS_OK;
  }
  if (!std::strcmp(key, "overlap_chunks")) {
    *value = ctx->overlap_chunks;
    return HERS_OK;
  }
  if (!std::strcmp(key, "mac_wgs_per_cu")) {
    *value = ctx->mac_wgs_per_cu;
    return HERS_OK;
  }
  if (!std::strcmp(key, "relin_fuse_min_wgs")) {
    *value = ctx->relin_fuse_min_wgs;
    return HERS_OK;
  }
  if (!std::strcmp(key, "mb_variant")) {
    *value = ctx->mb_variant;
    return HERS_OK;
  }
  if (!std::strcmp(key, "mb_group")) {
    *value = ctx->mb_group;
    return HERS_OK;
  }
  return fail(HERS_EINVAL, std::string("unknown option ") + key);
}

int hers_profile_enable(hers_ctx* ctx, int on) {
  if (!ctx) return fail(HERS_EINVAL, "null argument");
  DeviceGuard g(ctx->device);
  for (auto& r : ctx->pending) {
    (void)hipEventSynchronize(r.b);
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->pending.clear();
  ctx->totals.clear();
  ctx->prof_on = on != 0;
  return HERS_OK;
}

int hers_profile_select(hers_ctx* ctx, const char* stages) {
  if (!ctx) return fail(HERS_EINVAL, "null argument");
  ctx->prof_sel.clear();
  if (!stages) return HERS_OK;
  std::string cur;
  for (const char* c = stages;; ++c) {
    if (*c == ',' || *c == '\0') {
      if (!cur.empty()) ctx->prof_sel.push_back(cur);
      cur.clear();
      if (!*c) break;
    } else if (*c != ' ') {
      cur.push_back(*c);
    }
  }
  return HERS_OK;
}

int hers_profile_read(hers_ctx* ctx, const char* stage, double* total_ms, uint64_t* launches) {
  if (!ctx || !stage || !total_ms || !launches) return fail(HERS_EINVAL, "null argument");
  DeviceGuard g(ctx->device);
  for (auto& r : ctx->pending) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    auto& t = ctx->totals[r.stage];
    t.first += ms;
    t.second += 1;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->pending.clear();
  auto it = ctx->totals.find(stage);
  *total_ms = it == ctx->totals.end() ? 0.0 : it->second.first;
  *launches = it == ctx->totals.end() ? 0 : it->second.second;
  return HERS_OK;
}

int hers_ctx_info(const hers_ctx* ctx, hers_info* out) {
  if (!ctx || !out) return fail(HERS_EINVAL, "null argument");
  *out = ctx->host.info;
  return HERS_OK;
}

uint64_t hers_blocks(const hers_ctx* ctx, int64_t m) {
  if (!ctx || m < 0) return 0;
  return (uint64_t)((m + ctx->host.C.n - 1) / ctx->host.C.n);
}

uint64_t hers_ct_words(const hers_ctx* ctx) { return ctx ? (uint64_t)2 * ctx->host.C.k * ctx->host.C.n : 0; }
uint64_t hers_pk_words(const hers_ctx* ctx) { return hers_ct_words(ctx); }
uint64_t hers_rlk_words(const hers_ctx* ctx) { return ctx ? (uint64_t)ctx->host.C.L * hers_ct_words(ctx) : 0; }

uint64_t hers_gallery_words(const hers_ctx* ctx, int64_t m, int32_t d) {
  if (!ctx || d < 1) return 0;
  const HersConsts& C = ctx->host.C;
  return hers_blocks(ctx, m) * C.K * (uint64_t)d * 2 * C.n;
}

uint64_t hers_probe_words(const hers_ctx* ctx, int32_t d) {
  if (!ctx || d < 1) return 0;
  const HersConsts& C = ctx->host.C;
  return (uint64_t)C.K * d * 2 * C.n;
}

uint64_t hers_workspace_bytes(const hers_ctx* ctx, int op, int64_t m, int32_t d) {
  if (!ctx) return 0;
  const HersConsts& C = ctx->host.C;
  const uint64_t M = hers_blocks(ctx, m);
  switch (op) {
    case 0: return M * enc_ws_per_block(C, d, false);
    case 1: return align256((size_t)d * 2 * C.k * C.n * 8);
    case 2: return M * search_ws_per_block(C);
    case 3: return decrypt_ws_fixed(C) + M * decrypt_ws_per_block(C);
    case 4: return (M + 1) * enc_ws_per_block(C, d, false);
    case 5: return M * (search_ws_per_block(C) + align256((size_t)2 * C.k * C.n * 8));
    case 6: return (uint64_t)m * (align256((size_t)C.n * 4) + align256((size_t)2 * C.k * C.n * 8));
    case 7: return (uint64_t)m * rerank_ws_per_ct(C);
    case 8: return decrypt_ws_fixed(C) + (uint64_t)m * (decrypt_ws_per_block(C) + align256((size_t)C.n * 4));
    case 9: return M * (uint64_t)C.K * d * 2 * C.n * 4;
    case 10: return align256((size_t)d * 2 * C.k * C.n * 8) + align256((size_t)2 * C.k * C.n * 8);
    default: return 0;
  }
}

int hers_keygen(hers_ctx* ctx, uint64_t seed, uint8_t* sk_dev, uint64_t* pk_dev, uint64_t* rlk_dev, void* stream) {
  if (!ctx || !sk_dev || !pk_dev || !rlk_dev) return fail(HERS_EINVAL, "null argument");
  DeviceGuard g(ctx->device);
  const HersConsts& C = ctx->host.C;
  TIMED(ctx, "keygen", S(stream), hers::launch_keygen(ctx->T, C.n, C.k, C.L, seed, sk_dev, pk_dev, rlk_dev, S(stream)));
  ctx->keys_loaded = true;
  return HERS_OK;
}

int hers_load_keys(hers_ctx* ctx, const uint64_t* pk_dev, const uint64_t* rlk_dev, void* stream) {
  if (!ctx || !pk_dev || !rlk_dev) return fail(HERS_EINVAL, "null argument");
  DeviceGuard g(ctx->device);
  const HersConsts& C = ctx->host.C;
  TIMED(ctx, "load_keys", S(stream), hers::launch_load_keys(ctx->T, C.n, C.k, C.L, pk_dev, rlk_dev, S(stream)));
  ctx->keys_loaded = true;
  return HERS_OK;
}

int hers_encrypt_gallery(hers_ctx* ctx, const int32_t* feats_dev, int64_t ld, int64_t m_total, int32_t d,
                         int64_t block0, int64_t nblocks, uint64_t seed, uint32_t* gallery_dev,
                         uint64_t* canon_dev, void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || !feats_dev || !gallery_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no public key loaded");
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m_total);
  if (m_total < 1 || block0 < 0 || nblocks < 1 || block0 + nblocks > M)
    return fail(HERS_EINVAL, "block range outside the gallery");
  const int64_t need_items = (m_total - block0 * (int64_t)C.n) < nblocks * (int64_t)C.n
                                 ? m_total - block0 * (int64_t)C.n : nblocks * (int64_t)C.n;
  if (ld < need_items) return fail(HERS_EINVAL, "feature row stride smaller than the items of the range");
  const size_t per = enc_ws_per_block(C, d, canon_dev != nullptr);
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one block");
  const int64_t chunk = (int64_t)(work_bytes / per);
  DeviceGuard g(ctx->device);
  if (int rc = check_features(ctx, feats_dev, ld, d, need_items, S(stream))) return rc;
  for (int64_t lo = block0; lo < block0 + nblocks; lo += chunk) {
    const int64_t nb = (lo + chunk < block0 + nblocks) ? chunk : block0 + nblocks - lo;
    uint32_t* pt = (uint32_t*)work_dev;
    uint64_t* canon = canon_dev ? canon_dev + (size_t)lo * d * 2 * C.k * C.n
                                : (uint64_t*)((char*)work_dev + align256((size_t)nb * d * C.n * 4));
    TIMED(ctx, "encode", S(stream), hers::launch_encode(ctx->T, C.n, feats_dev, ld, 0, m_total, block0 * (int64_t)C.n,
                                                        d, lo, nb, pt, S(stream)));
    TIMED(ctx, "encrypt", S(stream), hers::launch_encrypt(ctx->T, C.n, C.k, (uint32_t)(nb * d), pt, nullptr, d, lo, seed,
                                 HERS_DOMAIN_GALLERY, canon, S(stream)));
    TIMED(ctx, "lift", S(stream), hers::launch_lift(ctx->T, C.n, canon, (uint32_t)(nb * d), d, lo, gallery_dev, S(stream)));
    TIMED(ctx, "ntt_fwd", S(stream), hers::launch_ntt_p(ctx->T, C.n, gallery_dev + (size_t)lo * C.K * d * 2 * C.n,
                               (uint64_t)nb * C.K * d * 2, 2 * d, 0, S(stream)));
  }
  return HERS_OK;
}

int hers_enroll_append(hers_ctx* ctx, const int32_t* feats_dev, int64_t ld, int64_t k0, int64_t c, int32_t d,
                       uint64_t seed, uint64_t* canon_dev, uint32_t* gallery_dev, void* work_dev, size_t work_bytes,
                       void* stream) {
  if (!ctx || !feats_dev || !canon_dev || !gallery_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no public key loaded");
  if (k0 < 0 || c < 1) return fail(HERS_EINVAL, "need k0 >= 0 and c >= 1");
  if (ld < c) return fail(HERS_EINVAL, "feature row stride smaller than the batch");
  const HersConsts& C = ctx->host.C;
  const int64_t n = C.n;
  const int64_t b_lo = k0 / n, b_hi = (k0 + c - 1) / n + 1;   // blocks the batch touches
  const size_t per = enc_ws_per_block(C, d, false);
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one block");
  const int64_t chunk = (int64_t)(work_bytes / per);
  const int64_t first_empty = (k0 + n - 1) / n;               // blocks from here held no item
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  if (int rc = check_features(ctx, feats_dev, ld, d, c, s)) return rc;
  for (int64_t lo = b_lo; lo < b_hi; lo += chunk) {
    const int64_t nb = lo + chunk < b_hi ? chunk : b_hi - lo;
    const uint32_t nct = (uint32_t)(nb * d);
    uint32_t* pt = (uint32_t*)work_dev;
    uint64_t* fresh = (uint64_t*)((char*)work_dev + align256((size_t)nb * d * C.n * 4));
    uint64_t* run = canon_dev + (size_t)lo * d * 2 * C.k * C.n;
    TIMED(ctx, "encode", s, hers::launch_encode(ctx->T, C.n, feats_dev, ld, k0, k0 + c, k0, d, lo, nb, pt, s));
    TIMED(ctx, "encrypt", s, hers::launch_encrypt(ctx->T, C.n, C.k, nct, pt, nullptr, d, lo, seed,
                                                  HERS_DOMAIN_ENROLL, fresh, s));
    TIMED(ctx, "ct_add", s, hers::launch_ct_add(ctx->T, C.n, C.k, run, fresh, nct, d, lo, first_empty, s));
    TIMED(ctx, "lift", s, hers::launch_lift(ctx->T, C.n, run, nct, d, lo, gallery_dev, s));
    TIMED(ctx, "ntt_fwd", s, hers::launch_ntt_p(ctx->T, C.n, gallery_dev + (size_t)lo * C.K * d * 2 * C.n,
                                                (uint64_t)nb * C.K * d * 2, 2 * d, 0, s));
  }
  return HERS_OK;
}

}  // extern "C"

// Query values (host) within +-feature_bound.
static int check_query(const hers_ctx* c, const int32_t* query, int32_t d) {
  const int64_t b = c->prm.feature_bound;
  for (int32_t i = 0; i < d; ++i)
    if ((int64_t)query[i] > b || (int64_t)query[i] < -b)
      return fail(HERS_ERANGE, "a query value lies outside [-feature_bound, feature_bound]");
  return HERS_OK;
}

// Probe encryption after the query's range check; the query (host) travels
// in the kernel arguments.
static int encrypt_probe_impl(hers_ctx* ctx, const int32_t* query, int32_t d, uint64_t seed, uint32_t* probe_dev,
                              uint64_t* canon_dev, void* work_dev, size_t work_bytes, hipStream_t s) {
  const HersConsts& C = ctx->host.C;
  uint64_t* canon = canon_dev;
  if (!canon) {
    if (!work_dev || work_bytes < (size_t)d * 2 * C.k * C.n * 8) return fail(HERS_ESPACE, "workspace too small");
    canon = (uint64_t*)work_dev;
  }
  DeviceGuard g(ctx->device);
  TIMED(ctx, "encrypt", s, hers::launch_encrypt(ctx->T, C.n, C.k, (uint32_t)d, nullptr, query, d, 0, seed,
                                                HERS_DOMAIN_PROBE, canon, s));
  TIMED(ctx, "lift", s, hers::launch_lift(ctx->T, C.n, canon, (uint32_t)d, d, 0, probe_dev, s));
  TIMED(ctx, "ntt_fwd", s, hers::launch_ntt_p(ctx->T, C.n, probe_dev, (uint64_t)C.K * d * 2, 2 * d, 0, s));
  return HERS_OK;
}

int hers::encrypt_probe_prechecked(hers_ctx* ctx, const int32_t* query, int32_t d, uint64_t seed,
                                   uint32_t* probe_dev, void* work_dev, size_t work_bytes, hipStream_t s) {
  if (!ctx || !query || !probe_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no public key loaded");
  return encrypt_probe_impl(ctx, query, d, seed, probe_dev, nullptr, work_dev, work_bytes, s);
}

extern "C" {

int hers_encrypt_probe(hers_ctx* ctx, const int32_t* query, int32_t d, uint64_t seed, uint32_t* probe_dev,
                       uint64_t* canon_dev, void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || !query || !probe_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no public key loaded");
  if (!canon_dev && (!work_dev || work_bytes < (size_t)d * 2 * ctx->host.C.k * ctx->host.C.n * 8))
    return fail(HERS_ESPACE, "workspace too small");
  if (int rc = check_query(ctx, query, d)) return rc;
  return encrypt_probe_impl(ctx, query, d, seed, probe_dev, canon_dev, work_dev, work_bytes, S(stream));
}

int hers_encrypt_probe_sk(hers_ctx* ctx, const uint8_t* sk_dev, const int32_t* query, int32_t d, uint64_t seed,
                          uint32_t* probe_dev, uint64_t probe_words, uint64_t* canon_dev, void* work_dev,
                          size_t work_bytes, void* stream) {
  if (!ctx || !query || !probe_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (!sk_dev && !ctx->sk_loaded) return fail(HERS_EINVAL, "no secret key given or loaded");
  const HersConsts& C = ctx->host.C;
  if (probe_words != (uint64_t)C.K * d * 2 * C.n)
    return fail(HERS_EDIM, "probe buffer length is not the search form of d dimensions");
  const size_t canon_b = canon_dev ? 0 : align256((size_t)d * 2 * C.k * C.n * 8);
  const size_t key_b = sk_dev ? align256((size_t)2 * C.k * C.n * 8) : 0;
  if (canon_b + key_b && (!work_dev || work_bytes < canon_b + key_b)) return fail(HERS_ESPACE, "workspace too small");
  if (int rc = check_query(ctx, query, d)) return rc;
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  uint64_t* canon = canon_dev ? canon_dev : (uint64_t*)work_dev;
  uint64_t* Sn = sk_dev ? (uint64_t*)((char*)work_dev + canon_b) : ctx->sk_ntt;
  uint64_t* Ssh = Sn + (size_t)C.k * C.n;
  if (sk_dev) TIMED(ctx, "sk_ntt", s, hers::launch_sk_ntt(ctx->T, C.n, C.k, sk_dev, Sn, Ssh, s));
  TIMED(ctx, "encrypt", s, hers::launch_encrypt_sk(ctx->T, C.n, C.k, query, d, seed, Sn, Ssh, canon, s));
  TIMED(ctx, "lift", s, hers::launch_lift(ctx->T, C.n, canon, (uint32_t)d, d, 0, probe_dev, s));
  TIMED(ctx, "ntt_fwd", s, hers::launch_ntt_p(ctx->T, C.n, probe_dev, (uint64_t)C.K * d * 2, 2 * d, 0, s));
  return HERS_OK;
}

// ---- canonical ciphertexts in and out of the search form
static int import_cts(hers_ctx* ctx, const uint64_t* canon_dev, int32_t d, int64_t block0, int64_t nblocks,
                      uint32_t* out, hipStream_t s) {
  const HersConsts& C = ctx->host.C;
  const uint64_t nct = (uint64_t)nblocks * d;
  if (nct > 0xffffffffull / C.n) return fail(HERS_EINVAL, "too many ciphertexts in one call");
  DeviceGuard g(ctx->device);
  if (int rc = flag_check(ctx, s, [&] {
        return hers::launch_check_canon(ctx->T, canon_dev, nct * 2 * C.k * C.n, ctx->flag_dev,
                                        (uint32_t)ctx->num_cus, s);
      }, HERS_ERANGE, "a canonical residue is not below its prime"))
    return rc;
  TIMED(ctx, "lift", s, hers::launch_lift(ctx->T, C.n, canon_dev, (uint32_t)nct, d, block0, out, s));
  TIMED(ctx, "ntt_fwd", s, hers::launch_ntt_p(ctx->T, C.n, out + (size_t)block0 * C.K * d * 2 * C.n,
                                              (uint64_t)nblocks * C.K * d * 2, 2 * d, 0, s));
  return HERS_OK;
}

int hers_import_gallery(hers_ctx* ctx, const uint64_t* canon_dev, int64_t m_total, int32_t d, int64_t block0,
                        int64_t nblocks, uint32_t* gallery_dev, uint64_t gallery_words, void* stream) {
  if (!ctx || !canon_dev || !gallery_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m_total);
  if (m_total < 1 || block0 < 0 || nblocks < 1 || block0 + nblocks > M)
    return fail(HERS_EINVAL, "block range outside the gallery");
  if (int rc = check_search_buffers(ctx, m_total, d, gallery_words, (uint64_t)C.K * d * 2 * C.n)) return rc;
  return import_cts(ctx, canon_dev, d, block0, nblocks, gallery_dev, S(stream));
}

int hers_import_probe(hers_ctx* ctx, const uint64_t* canon_dev, int32_t d, uint32_t* probe_dev, uint64_t probe_words,
                      void* stream) {
  if (!ctx || !canon_dev || !probe_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  const HersConsts& C = ctx->host.C;
  if (probe_words != (uint64_t)C.K * d * 2 * C.n)
    return fail(HERS_EDIM, "probe buffer length is not the search form of d dimensions");
  return import_cts(ctx, canon_dev, d, 0, 1, probe_dev, S(stream));
}

static int export_cts(hers_ctx* ctx, const uint32_t* search, int32_t d, int64_t nblocks, uint64_t* canon,
                      void* work_dev, size_t work_bytes, hipStream_t s) {
  const HersConsts& C = ctx->host.C;
  const size_t per = (size_t)C.K * d * 2 * C.n * 4;
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one block");
  const int64_t chunk = (int64_t)(work_bytes / per);
  DeviceGuard g(ctx->device);
  for (int64_t lo = 0; lo < nblocks; lo += chunk) {
    const int64_t nb = lo + chunk < nblocks ? chunk : nblocks - lo;
    uint32_t* coef = (uint32_t*)work_dev;
    HIP_TRY(hipMemcpyAsync(coef, search + (size_t)lo * C.K * d * 2 * C.n, (size_t)nb * per, hipMemcpyDeviceToDevice, s));
    TIMED(ctx, "ntt_inv", s, hers::launch_ntt_p(ctx->T, C.n, coef, (uint64_t)nb * C.K * d * 2, 2 * d, 1, s));
    TIMED(ctx, "unlift", s, hers::launch_unlift(ctx->T, C.n, coef, (uint32_t)(nb * d), d,
                                                canon + (size_t)lo * d * 2 * C.k * C.n, s));
  }
  return HERS_OK;
}

int hers_export_gallery(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m_total, int32_t d,
                        int64_t block0, int64_t nblocks, uint64_t* canon_dev, void* work_dev, size_t work_bytes,
                        void* stream) {
  if (!ctx || !gallery_dev || !canon_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m_total);
  if (m_total < 1 || block0 < 0 || nblocks < 1 || block0 + nblocks > M)
    return fail(HERS_EINVAL, "block range outside the gallery");
  if (int rc = check_search_buffers(ctx, m_total, d, gallery_words, (uint64_t)C.K * d * 2 * C.n)) return rc;
  if ((uint64_t)nblocks * d > 0xffffffffull / C.n) return fail(HERS_EINVAL, "too many ciphertexts in one call");
  return export_cts(ctx, gallery_dev + (size_t)block0 * C.K * d * 2 * C.n, d, nblocks, canon_dev, work_dev,
                    work_bytes, S(stream));
}

int hers_export_probe(hers_ctx* ctx, const uint32_t* probe_dev, uint64_t probe_words, int32_t d, uint64_t* canon_dev,
                      void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || !probe_dev || !canon_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  const HersConsts& C = ctx->host.C;
  if (probe_words != (uint64_t)C.K * d * 2 * C.n)
    return fail(HERS_EDIM, "probe buffer length is not the search form of d dimensions");
  return export_cts(ctx, probe_dev, d, 1, canon_dev, work_dev, work_bytes, S(stream));
}

// Relinearization launches with at least this many workgroups use the fused
// kernel.  Default: 8 per CU at n >= 8192 (measured faster there: each
// transformed digit saved is 64 KB).  Below n = 8192, the double-precision
// form of 8 coefficients per lane, whose transforms run their first and last
// passes in registers, measured 15-27% faster than the two-kernel form at
// every launch size at n = 4096 (16 to 4096 blocks), so it is always used
// where it applies (primes below 2^45, passes of at least 3 stages); other
// parameter sets below n = 8192 keep the two-kernel form.
static uint32_t fuse_wgs(const hers_ctx* ctx) {
  if (ctx->relin_fuse_min_wgs) return (uint32_t)ctx->relin_fuse_min_wgs;
  if (ctx->host.C.n >= 8192) return 8u * (uint32_t)ctx->num_cus;
  const bool edge_form = ctx->T.qf_ok && ctx->T.rl_per == 8 && ctx->T.ntt_r >= 3 && ctx->host.C.n >= 128;
  return edge_form ? 1u : 0xffffffffu;
}

static bool mac_fused(const hers_ctx* ctx) { return ctx->mac_variant == MAC_FUSED_INTT; }

// Workgroups of a multiply-accumulate launch.
static uint32_t mac_grid(const hers_ctx* ctx) {
  return (uint32_t)(ctx->mac_wgs_per_cu ? ctx->mac_wgs_per_cu : 8) * (uint32_t)ctx->num_cus;
}

// One probe's multiply-accumulate over blocks [lo, hi) (dimensions dim0 ..
// dim0 + dcount - 1, all for dcount 0) with schedule `variant`; the fused
// schedule leaves the accumulators in the coefficient domain.
static hipError_t launch_mac_sched(hers_ctx* ctx, int variant, const uint32_t* gallery, const uint32_t* probe,
                                   int32_t d, int64_t lo, int64_t hi, uint32_t* acc, hipStream_t s, int32_t dim0 = 0,
                                   int32_t dcount = 0) {
  const HersConsts& C = ctx->host.C;
  if (variant == MAC_FUSED_INTT) {
    // default: as many n/4-lane workgroups as fill a CU at 8 waves per SIMD
    const uint32_t lanes = C.n / 4, per_cu = ctx->mac_wgs_per_cu ? (uint32_t)ctx->mac_wgs_per_cu
                                                                  : (2048u / lanes > 0 ? 2048u / lanes : 1u);
    return hers::launch_mac_intt(ctx->T, C.n, C.K, gallery, probe, d, lo, hi, acc, s, per_cu * (uint32_t)ctx->num_cus,
                                 dim0, dcount);
  }
  return hers::launch_mac(ctx->T, C.n, C.K, gallery, probe, d, lo, hi, acc, s, variant, mac_grid(ctx), dim0, dcount);
}

// Per-block epilogue of blocks [lo, hi): inverse NTT of the accumulators
// (unless acc_coef: the multiply-accumulate left them in the coefficient
// domain), exact rescale (with the relinearization digits), relinearization.
static int search_epilogue(hers_ctx* ctx, uint32_t* acc, uint64_t* digits, int64_t lo, int64_t hi,
                           uint64_t* scores_dev, hipStream_t s, bool acc_coef) {
  const HersConsts& C = ctx->host.C;
  const int64_t nb = hi - lo;
  if (!acc_coef)
    TIMED(ctx, "intt_acc", s, hers::launch_ntt_p(ctx->T, C.n, acc, (uint64_t)nb * 3 * C.K, 1, 1, s));
  ScorePtrs sp;
  sp.p[0] = scores_dev;
  TIMED(ctx, "rescale", s,
        hers::launch_rescale(ctx->T, C.n, acc, nb, lo, sp, 1, digits, 0, 0, s, C.k, C.K, C.fr_words));
  TIMED(ctx, "relin", s, hers::launch_relin(ctx->T, C.n, C.k, C.L, digits, nb, lo, sp, 1, 0, s, nullptr, nullptr,
                                            fuse_wgs(ctx)));
  return HERS_OK;
}

}  // extern "C"

// The search (hers_search): blocks in chunks of the workspace; `overlap`
// allows the chunked schedule whose epilogues run on the context's second
// stream (it creates events on first use).
int hers::search_impl(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                      const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev, void* work_dev,
                      size_t work_bytes, void* stream, bool overlap) {
  if (!ctx || !gallery_dev || !probe_dev || !scores_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (m < 1) return fail(HERS_EINVAL, "empty gallery");
  if (int rc = check_search_buffers(ctx, m, d, gallery_words, probe_words)) return rc;
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no evaluation key loaded");
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m);
  const size_t per = search_ws_per_block(C);
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one block");
  const int64_t cap = (int64_t)(work_bytes / per);
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  int64_t nch = overlap ? ctx->overlap_chunks : 1;
  if (nch == 0) nch = M >= 4096 ? 8 : 1;
  if (nch <= 1 || cap < 2) {
    for (int64_t lo = 0; lo < M; lo += cap) {
      const int64_t hi = lo + cap < M ? lo + cap : M;
      uint32_t* acc = (uint32_t*)work_dev;
      uint64_t* digits = (uint64_t*)((char*)work_dev + align256((size_t)(hi - lo) * 3 * C.K * C.n * 4));
      TIMED(ctx, "mac", s, launch_mac_sched(ctx, ctx->mac_variant, gallery_dev, probe_dev, d, lo, hi, acc, s));
      if (int rc = search_epilogue(ctx, acc, digits, lo, hi, scores_dev, s, mac_fused(ctx))) return rc;
    }
    return HERS_OK;
  }
  // Overlapped: the blocks go in chunks of `sub`; chunk c's multiply-accumulate
  // runs on the caller's stream into workspace region c mod nreg, its epilogue
  // on the side stream, so the epilogue of one chunk (VALU-bound) runs beside
  // the next chunk's multiply-accumulate (HBM-bound).  A chunk waits for the
  // epilogue that last used its region; the caller's stream waits for the
  // side stream before the call returns.
  int64_t sub = (M + nch - 1) / nch;
  if (sub > cap / 2) sub = cap / 2;
  const int64_t nreg = std::min<int64_t>(cap / sub, (M + sub - 1) / sub);
  while ((int64_t)ctx->ev_free.size() < nreg) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->ev_free.push_back(e);
  }
  const size_t region = (size_t)sub * per;
  int rc = HERS_OK;
  hipError_t e = hipSuccess;
  for (int64_t c = 0, lo = 0; lo < M && rc == HERS_OK && e == hipSuccess; ++c, lo += sub) {
    const int64_t hi = lo + sub < M ? lo + sub : M;
    const int64_t r = c % nreg;
    char* base = (char*)work_dev + (size_t)r * region;
    uint32_t* acc = (uint32_t*)base;
    uint64_t* digits = (uint64_t*)(base + align256((size_t)(hi - lo) * 3 * C.K * C.n * 4));
    if (c >= nreg) e = hipStreamWaitEvent(s, ctx->ev_free[r], 0);
    if (e != hipSuccess) break;
    {
      StageTimer st(ctx, "mac", s);
      e = launch_mac_sched(ctx, ctx->mac_variant, gallery_dev, probe_dev, d, lo, hi, acc, s);
    }
    if (e == hipSuccess) e = hipEventRecord(ctx->ev_mac, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(ctx->side, ctx->ev_mac, 0);
    if (e != hipSuccess) break;
    rc = search_epilogue(ctx, acc, digits, lo, hi, scores_dev, ctx->side, mac_fused(ctx));
    if (rc == HERS_OK) e = hipEventRecord(ctx->ev_free[r], ctx->side);
  }
  // join even after a failure, so nothing of this call is left unordered
  hipError_t ej = hipEventRecord(ctx->ev_join, ctx->side);
  if (ej == hipSuccess) ej = hipStreamWaitEvent(s, ctx->ev_join, 0);
  if (rc != HERS_OK) return rc;
  if (e != hipSuccess) return fail(HERS_EDEVICE, std::string("overlapped search: ") + hipGetErrorString(e));
  if (ej != hipSuccess) return fail(HERS_EDEVICE, std::string("overlapped search join: ") + hipGetErrorString(ej));
  return HERS_OK;
}

int hers::ctx_device(const hers_ctx* ctx) { return ctx->device; }

size_t hers::search_ws_block_bytes(const hers_ctx* ctx) { return search_ws_per_block(ctx->host.C); }

extern "C" {

int hers_search(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev, void* work_dev,
                size_t work_bytes, void* stream) {
  return hers::search_impl(ctx, gallery_dev, gallery_words, m, d, probe_dev, probe_words, scores_dev, work_dev,
                           work_bytes, stream, true);
}

int hers_search_literal(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                        const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev, void* work_dev,
                        size_t work_bytes, void* stream) {
  if (!ctx || !gallery_dev || !probe_dev || !scores_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (m < 1) return fail(HERS_EINVAL, "empty gallery");
  if (int rc = check_search_buffers(ctx, m, d, gallery_words, probe_words)) return rc;
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no evaluation key loaded");
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m);
  const size_t ct_bytes = align256((size_t)2 * C.k * C.n * 8);
  const size_t per = search_ws_per_block(C) + ct_bytes;
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one block");
  const int64_t cap = (int64_t)(work_bytes / per);
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  for (int64_t lo = 0; lo < M; lo += cap) {
    const int64_t hi = lo + cap < M ? lo + cap : M;
    const int64_t nb = hi - lo;
    uint32_t* acc = (uint32_t*)work_dev;
    uint64_t* digits = (uint64_t*)((char*)work_dev + align256((size_t)nb * 3 * C.K * C.n * 4));
    uint64_t* prod = (uint64_t*)((char*)work_dev + (size_t)nb * search_ws_per_block(C));
    ScorePtrs sp;
    sp.p[0] = prod;                                   // indexed from block lo (blk_lo 0 below)
    for (int32_t i = 0; i < d; ++i) {
      // CipherMultiply(probe_i, gallery_i): tensor, rescale, relinearization ...
      TIMED(ctx, "mac", s, launch_mac_sched(ctx, ctx->mac_variant, gallery_dev, probe_dev, d, lo, hi, acc, s, i, 1));
      if (!mac_fused(ctx))
        TIMED(ctx, "intt_acc", s, hers::launch_ntt_p(ctx->T, C.n, acc, (uint64_t)nb * 3 * C.K, 1, 1, s));
      TIMED(ctx, "rescale", s,
            hers::launch_rescale(ctx->T, C.n, acc, nb, 0, sp, 1, digits, 0, 0, s, C.k, C.K, C.fr_words));
      TIMED(ctx, "relin", s, hers::launch_relin(ctx->T, C.n, C.k, C.L, digits, nb, 0, sp, 1, 0, s, nullptr, nullptr,
                                                fuse_wgs(ctx)));
      // ... then CipherAdd into the block's score (the first product starts it)
      TIMED(ctx, "ct_add", s, hers::launch_ct_add(ctx->T, C.n, C.k, scores_dev + (size_t)lo * 2 * C.k * C.n, prod,
                                                  (uint32_t)nb, 1, 0, i == 0 ? 0 : INT64_MAX, s));
    }
  }
  return HERS_OK;
}

static int log2_pow2(int32_t W) {
  int l = 0;
  while ((1 << l) < W) ++l;
  return (1 << l) == W ? l : -1;
}

static int check_w(const hers_ctx* ctx, int32_t W) {
  const int l = log2_pow2(W);
  if (l < 1 || W > (int32_t)(ctx->host.C.n / 2)) return fail(HERS_EINVAL, "W must be a power of two in [2, n/2]");
  return HERS_OK;
}

uint64_t hers_rotation_key_words(const hers_ctx* ctx, int32_t W) {
  if (!ctx || log2_pow2(W) < 1) return 0;
  return (uint64_t)log2_pow2(W) * ctx->host.C.L * 2 * ctx->host.C.k * ctx->host.C.n;
}

int hers_rotation_keygen(hers_ctx* ctx, uint64_t seed, int32_t W, uint64_t* rk_dev, void* stream) {
  if (!ctx || !rk_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_w(ctx, W)) return rc;
  const HersConsts& C = ctx->host.C;
  const int steps = log2_pow2(W);
  DeviceGuard g(ctx->device);
  if (!ctx->rk_ntt) {
    // room for every step up to W = n/2 (a setup call: the keys live in the context)
    const size_t bytes = (size_t)log2_pow2((int32_t)C.n / 2) * C.L * 2 * C.k * C.n * 8;
    if (hipMalloc((void**)&ctx->rk_ntt, bytes) != hipSuccess ||
        hipMalloc((void**)&ctx->rk_ntt_sh, bytes) != hipSuccess)
      return fail(HERS_ENOMEM, "hipMalloc of rotation keys failed");
  }
  TIMED(ctx, "keygen", S(stream), hers::launch_rotkey(ctx->T, C.n, C.k, C.L, (uint32_t)steps, seed, rk_dev,
                                                      ctx->rk_ntt, ctx->rk_ntt_sh, S(stream)));
  ctx->rk_steps = steps;
  return HERS_OK;
}

int hers_rerank_encrypt(hers_ctx* ctx, const int32_t* feats_dev, int64_t ld, int64_t count, int32_t D, int32_t W,
                        int replicate, uint64_t seed, uint32_t* search_dev, uint64_t* canon_dev, void* work_dev,
                        size_t work_bytes, void* stream) {
  if (!ctx || !feats_dev || !search_dev) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_w(ctx, W)) return rc;
  if (int rc = check_d(ctx, D)) return rc;
  if (D > W) return fail(HERS_EINVAL, "D must not exceed W");
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no public key loaded");
  if (count < 1 || (replicate && count != 1)) return fail(HERS_EINVAL, "count must be >= 1 (1 with replicate)");
  if (ld < count) return fail(HERS_EINVAL, "feature row stride smaller than count");
  const HersConsts& C = ctx->host.C;
  const int64_t S_ = C.n / W;
  const int64_t nct = replicate ? 1 : (count + S_ - 1) / S_;
  const size_t per = align256((size_t)C.n * 4) + (canon_dev ? 0 : align256((size_t)2 * C.k * C.n * 8));
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one ciphertext");
  const int64_t chunk = (int64_t)(work_bytes / per);
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  if (int rc = check_features(ctx, feats_dev, ld, D, count, s)) return rc;
  const uint32_t domain = replicate ? HERS_DOMAIN_RERANK_PROBE : HERS_DOMAIN_RERANK_ITEMS;
  for (int64_t lo = 0; lo < nct; lo += chunk) {
    const int64_t nb = lo + chunk < nct ? chunk : nct - lo;
    uint32_t* pt = (uint32_t*)work_dev;
    uint64_t* canon = canon_dev ? canon_dev + (size_t)lo * 2 * C.k * C.n
                                : (uint64_t*)((char*)work_dev + align256((size_t)nb * C.n * 4));
    const int32_t* f = replicate ? feats_dev : feats_dev + lo * S_;
    TIMED(ctx, "encode", s, hers::launch_encode_packed(ctx->T, C.n, f, ld, replicate ? 1 : count - lo * S_, D, W,
                                                       replicate, (uint32_t)nb, pt, s));
    TIMED(ctx, "encrypt", s, hers::launch_encrypt(ctx->T, C.n, C.k, (uint32_t)nb, pt, nullptr, 1, lo, seed, domain,
                                                  canon, s));
    TIMED(ctx, "lift", s, hers::launch_lift(ctx->T, C.n, canon, (uint32_t)nb, 1, lo, search_dev, s));
    TIMED(ctx, "ntt_fwd", s, hers::launch_ntt_p(ctx->T, C.n, search_dev + (size_t)lo * C.K * 2 * C.n,
                                                (uint64_t)nb * C.K * 2, 2, 0, s));
  }
  return HERS_OK;
}

int hers_rerank(hers_ctx* ctx, const uint32_t* items_search, int64_t nct_total, const int64_t* ids_dev, int32_t nsel,
                const uint32_t* probe_search, int32_t W, uint64_t* out_cts, void* work_dev, size_t work_bytes,
                void* stream) {
  if (!ctx || !items_search || !ids_dev || !probe_search || !out_cts) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_w(ctx, W)) return rc;
  if (nsel < 1 || nct_total < 1) return fail(HERS_EINVAL, "need nsel >= 1 and nct_total >= 1");
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no evaluation key loaded");
  const int steps = log2_pow2(W);
  if (ctx->rk_steps < steps) return fail(HERS_EINVAL, "rotation keys for this W not generated");
  const HersConsts& C = ctx->host.C;
  const size_t per = rerank_ws_per_ct(C);
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one ciphertext");
  int64_t cap = (int64_t)(work_bytes / per);
  if (cap > 65535) cap = 65535;
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  const size_t ct_words = (size_t)2 * C.k * C.n;
  const size_t key_words = (size_t)C.L * ct_words;
  for (int64_t lo = 0; lo < nsel; lo += cap) {
    const int64_t nb = lo + cap < nsel ? cap : nsel - lo;
    char* w = (char*)work_dev;
    uint32_t* gath = (uint32_t*)w;
    w += align256((size_t)nb * C.K * 2 * C.n * 4);
    uint32_t* acc = (uint32_t*)w;
    w += align256((size_t)nb * 3 * C.K * C.n * 4);
    uint64_t* digits = (uint64_t*)w;
    w += align256((size_t)nb * C.L * C.k * C.n * 8);
    uint64_t* tmp = (uint64_t*)w;
    TIMED(ctx, "gather", s, hers::launch_gather_cts(items_search, (uint64_t)C.K * 2 * C.n, nct_total, ids_dev + lo,
                                                   (uint32_t)nb, gath, s));
    // one ciphertext product per selected ciphertext (a search with d = 1)
    TIMED(ctx, "mac", s, launch_mac_sched(ctx, ctx->mac_variant, gath, probe_search, 1, 0, nb, acc, s));
    if (int rc = search_epilogue(ctx, acc, digits, 0, nb, out_cts + (size_t)lo * ct_words, s, mac_fused(ctx)))
      return rc;
    // rotate-and-add: cur -> nxt, ping-pong between out_cts and tmp
    uint64_t* cur = out_cts + (size_t)lo * ct_words;
    uint64_t* nxt = tmp;
    for (int st = 0; st < steps; ++st) {
      uint32_t gel = 5;
      for (int i = 0; i < st; ++i) gel = (gel * gel) & (2 * C.n - 1);
      TIMED(ctx, "rotate", s, hers::launch_rot_digits(ctx->T, C.n, C.k, cur, nxt, digits, (uint32_t)nb, gel, s));
      ScorePtrs sp;
      sp.p[0] = nxt;
      TIMED(ctx, "rotate", s, hers::launch_relin(ctx->T, C.n, C.k, C.L, digits, nb, 0, sp, 1, 0, s,
                                                 ctx->rk_ntt + (size_t)st * key_words,
                                                 ctx->rk_ntt_sh + (size_t)st * key_words, fuse_wgs(ctx)));
      std::swap(cur, nxt);
    }
    if (cur != out_cts + (size_t)lo * ct_words)
      HIP_TRY(hipMemcpyAsync(out_cts + (size_t)lo * ct_words, cur, (size_t)nb * ct_words * 8,
                             hipMemcpyDeviceToDevice, s));
  }
  return HERS_OK;
}

int hers_rerank_decrypt(hers_ctx* ctx, const uint8_t* sk_dev, const uint64_t* cts, int32_t nsel, int32_t W,
                        int32_t* scores_out, void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || !cts || !scores_out) return fail(HERS_EINVAL, "null argument");
  if (int rc = check_w(ctx, W)) return rc;
  if (nsel < 1) return fail(HERS_EINVAL, "need nsel >= 1");
  const HersConsts& C = ctx->host.C;
  const size_t slots_bytes = align256((size_t)nsel * C.n * 4);
  if (!work_dev || work_bytes < slots_bytes + decrypt_ws_fixed(C) + decrypt_ws_per_block(C))
    return fail(HERS_ESPACE, "workspace too small");
  DeviceGuard g(ctx->device);
  int32_t* slots = (int32_t*)work_dev;
  // decrypt every ciphertext as a block of n "items" (its slots), then pick
  // each segment's first position
  if (int rc = hers_decrypt_scores(ctx, sk_dev, cts, (int64_t)nsel * C.n, slots, (char*)work_dev + slots_bytes,
                                   work_bytes - slots_bytes, stream))
    return rc;
  TIMED(ctx, "dec_decode", S(stream), hers::launch_rerank_pick(C.n, slots, (uint32_t)nsel, W, scores_out, S(stream)));
  return HERS_OK;
}

int hers_autotune(hers_ctx* ctx, const uint32_t* gallery_dev, uint64_t gallery_words, int64_t m, int32_t d,
                  const uint32_t* probe_dev, uint64_t probe_words, uint64_t* scores_dev, void* work_dev,
                  size_t work_bytes, int reps, void* stream, int64_t* chosen) {
  if (!ctx || !gallery_dev || !probe_dev || reps < 1 || m < 1) return fail(HERS_EINVAL, "bad argument");
  if (int rc = check_d(ctx, d)) return rc;
  if (int rc = check_search_buffers(ctx, m, d, gallery_words, probe_words)) return rc;
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m);
  const size_t per = search_ws_per_block(C);
  if (!work_dev || work_bytes < per) return fail(HERS_ESPACE, "workspace smaller than one block");
  const int64_t hi = (int64_t)(work_bytes / per) < M ? (int64_t)(work_bytes / per) : M;
  DeviceGuard g(ctx->device);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 0.f, cur_ms = 0.f;
  int best_v = ctx->mac_variant;
  int rc = HERS_OK;
  // each schedule with the accumulators' inverse NTT (which the fused one does itself)
  const int nvar = C.n <= 4096 ? MAC_FUSED_INTT + 1 : MAC_FUSED_INTT;
  auto mac_intt = [&](int v) {
    uint32_t* acc = (uint32_t*)work_dev;
    hipError_t e = launch_mac_sched(ctx, v, gallery_dev, probe_dev, d, 0, hi, acc, S(stream));
    if (e == hipSuccess && v != MAC_FUSED_INTT)
      e = hers::launch_ntt_p(ctx->T, C.n, acc, (uint64_t)hi * 3 * C.K, 1, 1, S(stream));
    return e;
  };
  for (int v = 0; v < nvar && rc == HERS_OK; ++v) {
    hipError_t e = mac_intt(v);
    if (e == hipSuccess) e = hipEventRecord(e0, S(stream));
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = mac_intt(v);
    if (e == hipSuccess) e = hipEventRecord(e1, S(stream));
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { rc = fail(HERS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
    if (v == 0 || ms < best) { best = ms; best_v = v; }
    if (v == ctx->mac_variant) cur_ms = ms;
  }
  // keep the current schedule unless another is clearly faster (timing noise
  // between near-equal schedules would only make runs disagree)
  if (rc == HERS_OK && best > 0.97f * cur_ms) best_v = ctx->mac_variant;
  // NTT pass radix: time the search epilogue's transforms under radix 4, 8, 16:
  // inverse NTTs of the accumulators, then one block's relinearization (digit
  // NTTs, key products, inverse NTTs) writing into the accumulator area, which
  // holds 12 K n bytes per block, more than the 16 k n it writes (K > 2k).
  if (rc == HERS_OK) {
    uint32_t* acc = (uint32_t*)work_dev;
    uint64_t* digits = (uint64_t*)((char*)work_dev + align256((size_t)hi * 3 * C.K * C.n * 4));
    ScorePtrs sp;
    sp.p[0] = (uint64_t*)work_dev;
    float best_r = 0.f;
    uint32_t best_rl = ctx->T.ntt_r;
    for (uint32_t rl = 2; rl <= 4 && rc == HERS_OK; ++rl) {
      ctx->T.ntt_r = rl;
      hipError_t e = hipEventRecord(e0, S(stream));
      for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hers::launch_ntt_p(ctx->T, C.n, acc, (uint64_t)hi * 3 * C.K, 1, 1, S(stream));
        if (e == hipSuccess)
          e = hers::launch_relin(ctx->T, C.n, C.k, C.L, digits, 1, 0, sp, 1, 0, S(stream), nullptr, nullptr,
                                 fuse_wgs(ctx));
      }
      if (e == hipSuccess) e = hipEventRecord(e1, S(stream));
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) { rc = fail(HERS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e)); break; }
      if (rl == 2 || ms < best_r) { best_r = ms; best_rl = rl; }
    }
    ctx->T.ntt_r = best_rl;
  }
  if (rc == HERS_OK) ctx->mac_variant = best_v;
  // overlapped search: whole searches over chunk counts 1, 2, 4, ..., 64
  // (chunks of at least 16 blocks) x MAC workgroups per CU (default, 1, 2) x
  // the schedule chosen above, the default schedule 8 (the one timed alone
  // need not be the best beside the epilogue), schedule 10 (fewer registers,
  // so epilogue waves fit beside it), the fused schedule (n <= 4096) and
  // schedule 9 (two dimensions in flight per lane: more loads outstanding
  // from the few MAC waves a small grid leaves); then the fused
  // relinearization where the default is the two-kernel form.  The sweep
  // times each combination once (reps searches); the four fastest and the
  // plain one (no chunks, default grid, schedule found first) are then timed
  // again one search at a time in turn, 2 reps rounds, so that drift over
  // the sweep favours none of them, and the sums decide.
  if (rc == HERS_OK && scores_dev) {
    struct Cand { float ms; int nch, w, v; int64_t f; };
    std::vector<Cand> cands;
    const int64_t fuse0 = ctx->relin_fuse_min_wgs;
    auto apply = [&](const Cand& c) {
      ctx->overlap_chunks = c.nch;
      ctx->mac_wgs_per_cu = c.w;
      ctx->mac_variant = c.v;
      ctx->relin_fuse_min_wgs = c.f;
    };
    // one timed pass of `count` searches under c (after one untimed one when warm)
    auto time_searches = [&](const Cand& c, int count, bool warm, float* ms) -> int {
      apply(c);
      int r2 = warm ? hers_search(ctx, gallery_dev, gallery_words, m, d, probe_dev, probe_words, scores_dev,
                                  work_dev, work_bytes, stream)
                    : HERS_OK;
      hipError_t e = r2 == HERS_OK ? hipEventRecord(e0, S(stream)) : hipSuccess;
      for (int r = 0; r < count && r2 == HERS_OK && e == hipSuccess; ++r)
        r2 = hers_search(ctx, gallery_dev, gallery_words, m, d, probe_dev, probe_words, scores_dev, work_dev,
                         work_bytes, stream);
      if (r2 != HERS_OK) return r2;
      if (e == hipSuccess) e = hipEventRecord(e1, S(stream));
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
      if (e != hipSuccess) return fail(HERS_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
      return HERS_OK;
    };
    const int vs[5] = {best_v, 8, 10, nvar > MAC_FUSED_INTT ? MAC_FUSED_INTT : 10, 9};
    for (int nch = 1; nch <= 64 && rc == HERS_OK; nch *= 2) {
      if (nch > 1 && M / nch < 16) break;
      for (int w : {0, 1, 2}) {
        for (int vi = 0; vi < 5 && rc == HERS_OK; ++vi) {
          bool seen = false;
          for (int vj = 0; vj < vi; ++vj) seen |= vs[vj] == vs[vi];
          if (seen) continue;
          Cand c{0.f, nch, w, vs[vi], fuse0};
          rc = time_searches(c, reps, true, &c.ms);
          if (rc == HERS_OK) cands.push_back(c);
        }
      }
    }
    // the relinearization in one kernel per (block, prime) where the default
    // is the two-kernel form: it moves no transformed digit through memory,
    // which counts once the overlapped search is bound by its total traffic
    if (rc == HERS_OK && fuse_wgs(ctx) > 1 && !cands.empty()) {
      int mv = cands[0].v;
      float mb = cands[0].ms;
      for (const Cand& c : cands)
        if (c.ms < mb) { mb = c.ms; mv = c.v; }
      for (int nch : {1, 4, 16, 64}) {
        if (rc != HERS_OK || (nch > 1 && M / nch < 16)) break;
        for (int w : {0, 1}) {
          Cand c{0.f, nch, w, mv, 1};
          rc = time_searches(c, reps, true, &c.ms);
          if (rc == HERS_OK) cands.push_back(c);
        }
      }
    }
    if (rc == HERS_OK && !cands.empty()) {
      // cands[0] is the plain combination; the four fastest others join it
      std::vector<Cand> fin{cands[0]};
      std::vector<Cand> rest(cands.begin() + 1, cands.end());
      std::sort(rest.begin(), rest.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
      for (size_t i = 0; i < rest.size() && fin.size() < 5; ++i) fin.push_back(rest[i]);
      std::vector<float> tot(fin.size(), 0.f);
      for (int round = 0; round < 2 * reps && rc == HERS_OK; ++round)
        for (size_t i = 0; i < fin.size() && rc == HERS_OK; ++i) {
          float ms = 0.f;
          rc = time_searches(fin[i], 1, round == 0, &ms);
          tot[i] += ms;
        }
      if (rc == HERS_OK) {
        size_t bi = 0;
        for (size_t i = 1; i < fin.size(); ++i)
          if (tot[i] < tot[bi]) bi = i;
        // keep the plain combination unless another wins clearly: differences
        // within timing noise would only make runs disagree
        if (tot[bi] > 0.97f * tot[0]) bi = 0;
        apply(fin[bi]);
        best_v = fin[bi].v;
      }
    }
    if (rc != HERS_OK) {
      ctx->overlap_chunks = 1;
      ctx->mac_wgs_per_cu = 0;
      ctx->mac_variant = best_v;
      ctx->relin_fuse_min_wgs = fuse0;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (chosen) *chosen = best_v;
  return HERS_OK;
}

namespace {

struct BatchGroup {
  const uint32_t* gallery;
  int64_t m, M;
  int32_t d;
  std::vector<int32_t> reqs;
};

// Groups requests by (gallery, m, d), at most MB_PROBES per group.
int plan_groups(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries, const uint64_t* gallery_words,
                const int64_t* m, const int32_t* d, const uint32_t* const* probes, const uint64_t* probe_words,
                uint64_t* const* scores, std::vector<BatchGroup>* out) {
  out->clear();
  for (int32_t r = 0; r < nreq; ++r) {
    if (!galleries[r] || !probes[r] || !scores[r]) return fail(HERS_EINVAL, "null request pointer");
    if (int rc = check_d(ctx, d[r])) return rc;
    if (m[r] < 1) return fail(HERS_EINVAL, "empty gallery");
    if (int rc = check_search_buffers(ctx, m[r], d[r], gallery_words[r], probe_words[r])) return rc;
    BatchGroup* g = nullptr;
    for (auto& x : *out)
      if (x.gallery == galleries[r] && x.m == m[r] && x.d == d[r] && x.reqs.size() < (size_t)ctx->mb_group) {
        g = &x;
        break;
      }
    if (!g) {
      out->push_back({galleries[r], m[r], (int64_t)hers_blocks(ctx, m[r]), d[r], {}});
      g = &out->back();
    }
    g->reqs.push_back(r);
  }
  return HERS_OK;
}

// Enqueues a batch: rounds of at most CB blocks per group; per round one
// persistent multiply-accumulate launch per MB_MAXG groups, then the
// per-request epilogue (inverse NTT, rescale, relinearization).
// Workgroups per CU of a multi-probe schedule: as many as are resident.
uint32_t mb_wgs_per_cu(int variant) {
  static const uint32_t per_cu[MB_VARIANTS] = {1, 2, 2, 4, 1};
  return variant >= 0 && variant < MB_VARIANTS ? per_cu[variant] : 1;
}

// tune_variant >= 0: only the first round's multi-probe multiply-accumulate
// launches, with that schedule (the autotuner's timing run).
int run_batch(hers_ctx* ctx, const std::vector<BatchGroup>& groups, const uint32_t* const* probes,
              uint64_t* const* scores, void* work_dev, size_t work_bytes, hipStream_t s, int tune_variant = -1) {
  const HersConsts& C = ctx->host.C;
  size_t nprobe = 0;
  int64_t maxM = 0;
  for (auto& g : groups) { nprobe += g.reqs.size(); maxM = g.M > maxM ? g.M : maxM; }
  if (!nprobe) return HERS_OK;
  const size_t acc_pb = align256((size_t)3 * C.K * C.n * 4), dig_pb = align256((size_t)C.L * C.k * C.n * 8);
  int64_t CB = (int64_t)(work_bytes / (nprobe * (acc_pb + dig_pb)));
  if (!work_dev || CB < 1) return fail(HERS_ESPACE, "workspace smaller than one block per request");
  if (CB > MB_BLOCKS) CB = CB / MB_BLOCKS * MB_BLOCKS;
  char* base = (char*)work_dev;
  const size_t acc_bytes = nprobe * CB * acc_pb;
  const uint32_t tiles = C.n / 64;
  for (int64_t lo = 0; lo < maxM; lo += CB) {
    // accumulator slab per request, digits slab per request
    std::vector<uint32_t*> acc_of(groups.size());
    std::vector<uint64_t*> dig_of(groups.size());
    {
      size_t pi = 0;
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        acc_of[gi] = (uint32_t*)(base + pi * CB * acc_pb);
        dig_of[gi] = (uint64_t*)(base + acc_bytes + pi * CB * dig_pb);
        pi += groups[gi].reqs.size();
      }
    }
    MacBatchArgs A;
    std::memset(&A, 0, sizeof(A));
    auto flush = [&]() -> int {
      if (!A.ngroups) return HERS_OK;
      // the resident workgroups, a multiple of 8 (the kernel deals its items to the XCDs)
      const int v = tune_variant >= 0 ? tune_variant : ctx->mb_variant;
      uint64_t grid = (uint64_t)ctx->num_cus * mb_wgs_per_cu(v);
      if (grid > (A.total_items + 7) / 8 * 8) grid = (A.total_items + 7) / 8 * 8;
      TIMED(ctx, "mac_multi", s, hers::launch_mac_multi(ctx->T, A, (uint32_t)grid, s, v));
      std::memset(&A, 0, sizeof(A));
      return HERS_OK;
    };
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const BatchGroup& g = groups[gi];
      const int64_t hi = lo + CB < g.M ? lo + CB : g.M;
      if (lo >= hi) continue;
      if (g.reqs.size() == 1) {
        // a lone probe streams its gallery with the single-probe schedule
        if (tune_variant >= 0) continue;
        const int32_t r = g.reqs[0];
        TIMED(ctx, "mac", s, launch_mac_sched(ctx, ctx->mac_variant, g.gallery, probes[r], g.d, lo, hi, acc_of[gi],
                                              s));
        continue;
      }
      MacGroup& G = A.g[A.ngroups];
      G.gallery = g.gallery;
      for (size_t j = 0; j < g.reqs.size(); ++j) G.probe[j] = probes[g.reqs[j]];
      G.acc = acc_of[gi];
      G.acc_stride = CB * acc_pb / 4;
      G.blk_lo = lo;
      G.blk_hi = hi;
      G.item_begin = A.total_items;
      G.d = g.d;
      G.nprobe = (int32_t)g.reqs.size();
      A.total_items += (uint64_t)((hi - lo + MB_BLOCKS - 1) / MB_BLOCKS) * C.K * tiles;
      if (++A.ngroups == MB_MAXG)
        if (int rc = flush()) return rc;
    }
    if (int rc = flush()) return rc;
    if (tune_variant >= 0) return HERS_OK;
    // epilogue: the requests of a group share a block range; their slabs are
    // consecutive, so one launch per kernel covers up to EP_MAXR of them
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const BatchGroup& g = groups[gi];
      const int64_t hi = lo + CB < g.M ? lo + CB : g.M;
      if (lo >= hi) continue;
      const uint64_t as = CB * acc_pb / 4, ds = CB * dig_pb / 8;
      for (size_t j0 = 0; j0 < g.reqs.size(); j0 += EP_MAXR) {
        const uint32_t nr = (uint32_t)(g.reqs.size() - j0 < EP_MAXR ? g.reqs.size() - j0 : EP_MAXR);
        uint32_t* acc = acc_of[gi] + j0 * as;
        uint64_t* dig = dig_of[gi] + j0 * ds;
        ScorePtrs sp;
        for (uint32_t j = 0; j < nr; ++j) sp.p[j] = scores[g.reqs[j0 + j]];
        if (!(g.reqs.size() == 1 && mac_fused(ctx)))      // a lone probe's fused MAC left them transformed
          TIMED(ctx, "intt_acc", s,
                hers::launch_ntt_p(ctx->T, C.n, acc, (uint64_t)(hi - lo) * 3 * C.K, 1, 1, s, nr, as));
        TIMED(ctx, "rescale", s,
              hers::launch_rescale(ctx->T, C.n, acc, hi - lo, lo, sp, nr, dig, as, ds, s, C.k, C.K, C.fr_words));
        TIMED(ctx, "relin", s, hers::launch_relin(ctx->T, C.n, C.k, C.L, dig, hi - lo, lo, sp, nr, ds, s, nullptr,
                                                  nullptr, fuse_wgs(ctx)));
      }
    }
  }
  return HERS_OK;
}

}  // namespace

int hers_search_batch(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries, const uint64_t* gallery_words,
                      const int64_t* m, const int32_t* d, const uint32_t* const* probes, const uint64_t* probe_words,
                      uint64_t* const* scores, void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || nreq < 0 ||
      (nreq && (!galleries || !gallery_words || !m || !d || !probes || !probe_words || !scores)))
    return fail(HERS_EINVAL, "null argument");
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no evaluation key loaded");
  std::vector<BatchGroup> groups;
  if (int rc = plan_groups(ctx, nreq, galleries, gallery_words, m, d, probes, probe_words, scores, &groups)) return rc;
  DeviceGuard g(ctx->device);
  return run_batch(ctx, groups, probes, scores, work_dev, work_bytes, S(stream));
}

int hers_autotune_batch(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries, const uint64_t* gallery_words,
                        const int64_t* m, const int32_t* d, const uint32_t* const* probes, const uint64_t* probe_words,
                        uint64_t* const* scores, void* work_dev, size_t work_bytes, int reps, void* stream,
                        int64_t* chosen) {
  if (!ctx || nreq < 1 || reps < 1 || !galleries || !gallery_words || !m || !d || !probes || !probe_words || !scores)
    return fail(HERS_EINVAL, "bad argument");
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no evaluation key loaded");
  std::vector<BatchGroup> groups;
  if (int rc = plan_groups(ctx, nreq, galleries, gallery_words, m, d, probes, probe_words, scores, &groups)) return rc;
  bool multi = false;
  for (auto& g : groups) multi |= g.reqs.size() > 1;
  if (!multi) {                                       // nothing runs the multi-probe kernel
    if (chosen) *chosen = ctx->mb_variant;
    return HERS_OK;
  }
  DeviceGuard g(ctx->device);
  const hipStream_t s = S(stream);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 0.f, cur = 0.f;
  int best_v = ctx->mb_variant, rc = HERS_OK;
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  for (int v = 0; v < MB_VARIANTS && rc == HERS_OK; ++v) {
    rc = run_batch(ctx, groups, probes, scores, work_dev, work_bytes, s, v);      // warm-up
    hipError_t e = rc == HERS_OK ? hipEventRecord(e0, s) : hipSuccess;
    for (int r = 0; r < reps && rc == HERS_OK && e == hipSuccess; ++r)
      rc = run_batch(ctx, groups, probes, scores, work_dev, work_bytes, s, v);
    if (rc != HERS_OK) break;
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) { rc = fail(HERS_EDEVICE, std::string("autotune_batch: ") + hipGetErrorString(e)); break; }
    if (v == 0 || ms < best) { best = ms; best_v = v; }
    if (v == ctx->mb_variant) cur = ms;
  }
  ctx->prof_on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != HERS_OK) return rc;
  if (best > 0.97f * cur) best_v = ctx->mb_variant;   // keep the current one unless another is clearly faster
  ctx->mb_variant = best_v;
  if (chosen) *chosen = best_v;
  return HERS_OK;
}

struct hers_plan {
  hers_ctx* ctx;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int hers_plan_create(hers_ctx* ctx, int32_t nreq, const uint32_t* const* galleries, const uint64_t* gallery_words,
                     const int64_t* m, const int32_t* d, const uint32_t* const* probes, const uint64_t* probe_words,
                     uint64_t* const* scores, void* work_dev, size_t work_bytes, hers_plan** out) {
  if (!ctx || !out || nreq < 1 || !galleries || !gallery_words || !m || !d || !probes || !probe_words || !scores)
    return fail(HERS_EINVAL, "null argument");
  if (!ctx->keys_loaded) return fail(HERS_EINVAL, "no evaluation key loaded");
  *out = nullptr;
  std::vector<BatchGroup> groups;
  if (int rc = plan_groups(ctx, nreq, galleries, gallery_words, m, d, probes, probe_words, scores, &groups)) return rc;
  DeviceGuard g(ctx->device);
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;   // no event nodes in the graph
  hers_plan* p = new hers_plan{ctx};
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  int rc = e == hipSuccess ? run_batch(ctx, groups, probes, scores, work_dev, work_bytes, cs) : HERS_EDEVICE;
  hipError_t e2 = hipStreamEndCapture(cs, &p->graph);
  ctx->prof_on = prof;
  if (rc == HERS_OK && e == hipSuccess && e2 == hipSuccess)
    e2 = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (rc != HERS_OK || e != hipSuccess || e2 != hipSuccess) {
    std::string msg = rc != HERS_OK ? g_err : std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return fail(rc != HERS_OK ? rc : HERS_EDEVICE, msg);
  }
  *out = p;
  return HERS_OK;
}

int hers_plan_launch(hers_plan* plan, void* stream) {
  if (!plan) return fail(HERS_EINVAL, "null plan");
  DeviceGuard g(plan->ctx->device);
  HIP_TRY(hipGraphLaunch(plan->exec, S(stream)));
  return HERS_OK;
}

void hers_plan_destroy(hers_plan* plan) {
  if (!plan) return;
  DeviceGuard g(plan->ctx->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
}

int hers_load_secret_key(hers_ctx* ctx, const uint8_t* sk_dev, void* stream) {
  if (!ctx || !sk_dev) return fail(HERS_EINVAL, "null argument");
  const HersConsts& C = ctx->host.C;
  DeviceGuard g(ctx->device);
  if (!ctx->sk_ntt && hipMalloc((void**)&ctx->sk_ntt, (size_t)2 * C.k * C.n * 8) != hipSuccess)
    return fail(HERS_ENOMEM, "hipMalloc of the secret key form failed");
  TIMED(ctx, "sk_ntt", S(stream), hers::launch_sk_ntt(ctx->T, C.n, C.k, sk_dev, ctx->sk_ntt,
                                                      ctx->sk_ntt + (size_t)C.k * C.n, S(stream)));
  ctx->sk_loaded = true;
  return HERS_OK;
}

int hers_decrypt_scores(hers_ctx* ctx, const uint8_t* sk_dev, const uint64_t* scores_dev, int64_t m,
                        int32_t* scores_out_dev, void* work_dev, size_t work_bytes, void* stream) {
  if (!ctx || !scores_dev || !scores_out_dev) return fail(HERS_EINVAL, "null argument");
  if (!sk_dev && !ctx->sk_loaded) return fail(HERS_EINVAL, "no secret key given or loaded");
  if (m < 1) return fail(HERS_EINVAL, "empty gallery");
  const HersConsts& C = ctx->host.C;
  const int64_t M = (int64_t)hers_blocks(ctx, m);
  const size_t fixed = decrypt_ws_fixed(C), per = decrypt_ws_per_block(C);
  if (!work_dev || work_bytes < fixed + per) return fail(HERS_ESPACE, "workspace too small");
  const int64_t chunk = (int64_t)((work_bytes - fixed) / per);
  uint64_t* Sn = sk_dev ? (uint64_t*)work_dev : ctx->sk_ntt;
  uint64_t* Ssh = Sn + (size_t)C.k * C.n;
  uint64_t* x = (uint64_t*)((char*)work_dev + fixed);
  DeviceGuard g(ctx->device);
  if (sk_dev) TIMED(ctx, "sk_ntt", S(stream), hers::launch_sk_ntt(ctx->T, C.n, C.k, sk_dev, Sn, Ssh, S(stream)));
  if (hers::dec_fused_fits(ctx->T, C.n) && ctx->dec_fused) {
    // one kernel per block: x stays in registers (the workspace's x area is unused)
    TIMED(ctx, "decrypt", S(stream), hers::launch_dec_fused(ctx->T, C.n, scores_dev, M, 0, Sn, m, scores_out_dev,
                                                             S(stream)));
    return HERS_OK;
  }
  for (int64_t lo = 0; lo < M; lo += chunk) {
    const int64_t nb = lo + chunk < M ? chunk : M - lo;
    TIMED(ctx, "dec_mul", S(stream), hers::launch_dec_mul(ctx->T, C.n, C.k, scores_dev, nb, lo, Sn, Ssh, x, S(stream)));
    TIMED(ctx, "dec_decode", S(stream), hers::launch_dec_decode(ctx->T, C.n, x, nb, lo, m, scores_out_dev, S(stream)));
  }
  return HERS_OK;
}

}  // extern "C"
