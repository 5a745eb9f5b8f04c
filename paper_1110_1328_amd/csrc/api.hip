// C ABI entry points: argument validation, table cache, workspace, dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "device_common.h"

namespace blsh {

// launchers (verify.hip, sigs.hip)
int launch_verify(blsh_ctx *ctx, const VerifyArgs &a, int k, bool lite, bool word_major, hipStream_t s);
int launch_exhaustive(blsh_ctx *ctx, const VerifyArgs &a, int k, hipStream_t s);
int launch_zero(blsh_ctx *ctx, int64_t *p, hipStream_t s);
int launch_minhash(blsh_ctx *ctx, const int64_t *offsets, const uint32_t *elems, int64_t n_sets, const uint32_t *a,
                   const uint32_t *b, int n_hashes, uint32_t *out, hipStream_t s);
int launch_srp_sparse(blsh_ctx *ctx, const int64_t *offsets, const uint32_t *indices, const float *values,
                      int64_t n_rows, int64_t dim, int n_bits, uint64_t seed, bool word_major, bool q16,
                      uint32_t *out, hipStream_t s);
int launch_srp_dense(blsh_ctx *ctx, const float *X, int64_t n_rows, int64_t dim, const float *R, int n_bits,
                     bool word_major, uint32_t *out, hipStream_t s);

int launch_exact(blsh_ctx *ctx, const VerifyArgs &a, int64_t max_items, hipStream_t s);
int launch_exact_pairs(blsh_ctx *ctx, const VerifyArgs &a, double *out, hipStream_t s);
int launch_verify_tail(blsh_ctx *ctx, const VerifyArgs &a, int k, bool word_major, int words, hipStream_t s);
int launch_zero_slices(blsh_ctx *ctx, int64_t *cnt, hipStream_t s);
int launch_tiles_exact(blsh_ctx *ctx, const VerifyArgs &a, int64_t grid_waves, hipStream_t s);
int launch_verify_tiles(blsh_ctx *ctx, const VerifyArgs &a, int k, int n_max, int words, bool intervals, bool lite,
                        int64_t grid_waves, hipStream_t s);
int tiles_grid_waves(blsh_ctx *ctx, int k, int n_max, bool intervals, bool lite, size_t lds, int64_t *waves);
int launch_tiles_flush(blsh_ctx *ctx, const VerifyArgs &a, int64_t grid_waves, int64_t *off, bool last,
                       hipStream_t s);
int launch_acc_flush(blsh_ctx *ctx, const VerifyArgs &a, int64_t *nxt_cnt, int64_t *nxt_total, bool last,
                     hipStream_t s);
int band_candidates(blsh_ctx *ctx, const uint32_t *sig, int64_t n_obj, int32_t row_words, bool word_major,
                    int32_t n_bands, int32_t band_bits, int32_t max_bucket, int32_t tile, uint32_t *x_out,
                    uint32_t *y_out, int64_t capacity, int64_t *n_pairs, hipStream_t s, const BandTilesOut *to);
int verify_batched(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand, int64_t n_cand,
                   const blsh_sigs *jac, const blsh_sigs *cos, double eps, double delta, double gamma,
                   blsh_prior prior, int32_t kj, int32_t kc, blsh_result *res, int32_t *k_used, hipStream_t s,
                   int (*check_sigs_fn)(const blsh_sigs *, int, int *, int *), int mode);

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

LaunchScope::LaunchScope(blsh_ctx *c, hipStream_t s, const char *n) : ctx(c), stream(s), name(n), on(c && c->prof) {
  if (on) {
    hipEventCreate(&a);
    hipEventCreate(&b);
    hipEventRecord(a, stream);
  }
}
LaunchScope::~LaunchScope() {
  if (on) {
    hipEventRecord(b, stream);
    ctx->prof_pending.push_back({name, a, b});
  }
}

int get_table(blsh_ctx *ctx, const TableKey &key, std::shared_ptr<HostTable> *host, const uint32_t **dev,
              hipStream_t stream) {
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->host_tables.find(key);
  std::shared_ptr<HostTable> ht;
  if (it == ctx->host_tables.end()) {
    ht = std::make_shared<HostTable>();
    int rc = build_table(key, ht.get());
    if (rc != BLSH_OK) return rc;
    ctx->host_tables[key] = ht;
  } else {
    ht = it->second;
  }
  if (ht->image.empty()) {   // the device image of the table, kept with it
    std::vector<uint32_t> &img = ht->image;
    img.assign(kTabAccOff + size_t(ht->n_levels) * ht->words, 0u);
    img[0] = uint32_t(ht->k);
    img[1] = uint32_t(ht->n_levels);
    img[2] = uint32_t(ht->words);
    img[3] = uint32_t(key.measure);
    std::memcpy(&img[4], &key.alpha, 8);
    std::memcpy(&img[6], &key.beta, 8);
    std::memcpy(&img[8], &key.t, 8);
    bool intervals = true;
    for (int j = 0; j < ht->n_levels; ++j) {
      const int n = (j + 1) * ht->k, mm = ht->min_matches[j];
      img[kTabMinOff + j] = uint32_t(mm);
      // the accept set above min_matches: [lo, n] when it is an interval
      auto bit = [&](int m) { return (ht->accept[size_t(j) * ht->words + (m >> 5)] >> (m & 31)) & 1u; };
      int lo = n + 1;
      for (int m = n; m >= mm && m >= 0 && bit(m); --m) lo = m;
      for (int m = mm; m < lo; ++m)
        if (bit(m)) intervals = false;
      img[kTabAloOff + j] = uint32_t(lo);
    }
    img[kTabFlagOff] = intervals ? 1u : 0u;
    std::memcpy(&img[kTabAccOff], ht->accept.data(), ht->accept.size() * 4);
  }
  if (host) *host = ht;
  if (dev) {
    auto dt = ctx->dev_tables.find(key);
    if (dt == ctx->dev_tables.end()) {
      DevTable d;
      d.words = ht->image.size();
      BLSH_HIP(hipMalloc(&d.ptr, d.words * 4));
      BLSH_HIP(hipMemcpy(d.ptr, ht->image.data(), d.words * 4, hipMemcpyHostToDevice));
      dt = ctx->dev_tables.emplace(key, d).first;
    }
    *dev = dt->second.ptr;
  }
  (void)stream;
  return BLSH_OK;
}

int ensure_workspace(blsh_ctx *ctx, size_t bytes) {
  if (ctx->ws_bytes >= bytes) return BLSH_OK;
  if (ctx->ws_fixed)
    return fail(BLSH_ENOMEM, "the call needs %zu bytes of workspace; the context's is fixed at %zu", bytes,
                ctx->ws_bytes);
  BLSH_HIP(hipDeviceSynchronize());
  if (ctx->ws) hipFree(ctx->ws);
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  if (hipMalloc(&ctx->ws, bytes) != hipSuccess) {
    ctx->ws = nullptr;
    return fail(BLSH_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
  }
  ctx->ws_bytes = bytes;
  return BLSH_OK;
}

// ---------------------------------------------------------------------------
// validation helpers
// ---------------------------------------------------------------------------
static bool in01(double v) { return v > 0.0 && v < 1.0 && std::isfinite(v); }

static int check_params(double t, double eps, double delta, double gamma, bool lite) {
  if (!in01(t)) return fail(BLSH_EINVAL, "t must be in (0,1), got %g", t);
  if (!in01(eps)) return fail(BLSH_EINVAL, "epsilon must be in (0,1), got %g", eps);
  if (!lite && !in01(delta)) return fail(BLSH_EINVAL, "delta must be in (0,1), got %g", delta);
  if (!lite && !in01(gamma)) return fail(BLSH_EINVAL, "gamma must be in (0,1), got %g", gamma);
  return BLSH_OK;
}

static int check_prior(int measure, blsh_prior p) {
  if (measure == BLSH_COSINE) {
    if (p.alpha != 1.0 || p.beta != 1.0)
      return fail(BLSH_EINVAL, "cosine uses the uniform prior on r in [0.5,1]: prior must be {1,1}");
    return BLSH_OK;
  }
  if (!(p.alpha > 0.0 && p.beta > 0.0) || !(p.alpha <= 1e6 && p.beta <= 1e6))
    return fail(BLSH_EINVAL, "Jaccard prior Beta(alpha,beta) needs 0 < alpha, beta <= 1e6 (got %g,%g)", p.alpha,
                p.beta);
  return BLSH_OK;
}

static int check_sigs(const blsh_sigs *s, int k, int *n_max_out, int *row_words) {
  if (!s || !s->data) return fail(BLSH_EINVAL, "signatures: null");
  if (s->measure != BLSH_JACCARD && s->measure != BLSH_COSINE) return fail(BLSH_EINVAL, "signatures: bad measure");
  if (s->n_obj <= 0 || s->n_obj > 0xFFFFFFFFll) return fail(BLSH_EINVAL, "signatures: n_obj out of range");
  if (s->n_hashes <= 0) return fail(BLSH_EINVAL, "signatures: n_hashes <= 0");
  const int n_max = s->n_max ? s->n_max : s->n_hashes;
  if (n_max > s->n_hashes || n_max <= 0) return fail(BLSH_EINVAL, "signatures: n_max > n_hashes");
  if (k != 16 && k != 32 && k != 64) return fail(BLSH_EINVAL, "k must be 16, 32 or 64 (got %d)", k);
  if (n_max % k) return fail(BLSH_EINVAL, "n_max (%d) must be a multiple of k (%d)", n_max, k);
  if (n_max / k > kMaxLevels) return fail(BLSH_EINVAL, "n_max/k = %d levels exceeds %d", n_max / k, kMaxLevels);
  if (s->measure == BLSH_COSINE) {
    if (s->n_hashes % 32) return fail(BLSH_EINVAL, "SRP signatures: n_hashes must be a multiple of 32");
    if (s->layout != BLSH_OBJECT_MAJOR && s->layout != BLSH_WORD_MAJOR) return fail(BLSH_EINVAL, "bad layout");
    if (s->prefix && (s->n_hashes < 128 || (uintptr_t(s->prefix) & 15)))
      return fail(BLSH_EINVAL, "SRP prefix: needs n_hashes >= 128 and 16-byte alignment");
    *row_words = s->n_hashes / 32;
  } else {
    if (s->prefix) return fail(BLSH_EINVAL, "a prefix array is for SRP signatures only");
    if (s->layout != BLSH_OBJECT_MAJOR) return fail(BLSH_EINVAL, "minhash signatures must be OBJECT_MAJOR");
    if (s->n_hashes % 4) return fail(BLSH_EINVAL, "minhash signatures: n_hashes must be a multiple of 4");
    if (uintptr_t(s->data) & 15) return fail(BLSH_EINVAL, "minhash signatures must be 16-byte aligned");
    *row_words = s->n_hashes;
  }
  *n_max_out = n_max;
  return BLSH_OK;
}

int check_sigs_public(const blsh_sigs *s, int k, int *n_max_out, int *row_words) {
  return check_sigs(s, k, n_max_out, row_words);
}

static int check_cand(const blsh_candidates *c, int64_t *n_cand) {
  if (!c) return fail(BLSH_EINVAL, "candidates: null");
  switch (c->kind) {
    case BLSH_PAIRS:
      if (c->n_pairs < 0) return fail(BLSH_EINVAL, "candidates: n_pairs < 0");
      if (c->n_pairs && (!c->x || !c->y)) return fail(BLSH_EINVAL, "candidates: null x/y");
      *n_cand = c->n_pairs;
      return BLSH_OK;
    case BLSH_QUERY_LISTS:
      if (c->n_lists < 0 || c->n_cand < 0) return fail(BLSH_EINVAL, "candidates: negative list sizes");
      if (c->n_cand && (c->n_lists == 0 || !c->query || !c->offsets || !c->cand))
        return fail(BLSH_EINVAL, "candidates: null list arrays");
      *n_cand = c->n_cand;
      return BLSH_OK;
    case BLSH_ALL_PAIRS:
      if (c->all_n < 0 || c->all_n > (1ll << 31)) return fail(BLSH_EINVAL, "candidates: all_n out of range");
      *n_cand = c->all_n * (c->all_n - 1) / 2;
      if (c->all_n < 2) *n_cand = 0;
      return BLSH_OK;
    case BLSH_TILES:
      if (c->n_tiles < 0 || c->n_cand < 0) return fail(BLSH_EINVAL, "candidates: negative tile sizes");
      if (c->n_tiles > 0 && !c->tiles) return fail(BLSH_EINVAL, "candidates: null tiles");
      if (uintptr_t(c->tiles) & 15) return fail(BLSH_EINVAL, "candidates: tiles must be 16-byte aligned");
      *n_cand = c->n_cand;
      return BLSH_OK;
    default:
      return fail(BLSH_EINVAL, "candidates: bad kind %d", int(c->kind));
  }
}

static int check_result(const blsh_result *r) {
  if (!r || !r->code || !r->n_accepted) return fail(BLSH_EINVAL, "result: code and n_accepted are required");
  if (r->acc_capacity < 0) return fail(BLSH_EINVAL, "result: acc_capacity < 0");
  if (r->acc_capacity > 0 && (!r->acc_idx || !r->acc_val)) return fail(BLSH_EINVAL, "result: null acc arrays");
  return BLSH_OK;
}

static int check_exact(const blsh_vectors *v, int measure, int64_t n_obj) {
  if (!v) return fail(BLSH_EINVAL, "exact vectors: null");
  if (v->n_obj < n_obj) return fail(BLSH_EINVAL, "exact vectors: fewer objects than signatures");
  if (measure == BLSH_JACCARD) {
    if (v->kind != BLSH_SETS || !v->offsets || !v->indices)
      return fail(BLSH_EINVAL, "Jaccard exact similarity needs SETS vectors");
  } else if (v->kind == BLSH_DENSE) {
    if (!v->dense || v->dim <= 0) return fail(BLSH_EINVAL, "dense vectors: null or dim <= 0");
  } else if (v->kind == BLSH_CSR) {
    if (!v->offsets || !v->indices || !v->values) return fail(BLSH_EINVAL, "CSR vectors: null arrays");
  } else {
    return fail(BLSH_EINVAL, "cosine exact similarity needs DENSE or CSR vectors");
  }
  return BLSH_OK;
}

static void fill_cand(VerifyArgs &a, const blsh_candidates *c) {
  a.kind = c->kind;
  a.x = c->x;
  a.y = c->y;
  a.query = c->query;
  a.offsets = c->offsets;
  a.cand = c->cand;
  a.n_lists = c->n_lists;
  a.all_n = c->all_n;
}

// Buffers of one verify call, for launches of at most `chunk` candidates.
// Counters (the context's slice buffer), kCntStride int64 apart:
//   [0, S)           staging counts, set 0
//   [S, 2S)          staging counts, set 1
//   [2S, 3S)         survivor-queue counts
//   3S, 3S + 1       running accepted count of set 0, set 1
// Context workspace:
//   q_rel [, q_m]    kSlices survivor-queue slices of q_cap entries (q_m: the
//                    SRP tail's m | level << 16 beside each index): a launch
//                    of n candidates puts at most ceil((n + 1024) / kSlices) +
//                    256 entries in one slice (every kernel's waves take at most
//                    256 candidates and its blocks at most 1024, and wave w
//                    uses slice w % kSlices), so a slice never overflows
//   st_rel, st_val   kSlices accepted-pair staging slices of st_cap entries
static constexpr int64_t kChunk = int64_t(1) << 28;
static constexpr int64_t kExhChunk = int64_t(1) << 24;
static constexpr int64_t kStageDefault = int64_t(1) << 24;
static constexpr size_t kSliceBufWords = (size_t(3) * kSlices + 2) * kCntStride;

struct Workspace {
  int64_t *cnt;   // the context's counter buffer
  uint32_t *q_rel, *q_m;
  int64_t q_cap;
  uint32_t *st_rel;
  float *st_val;
  int64_t st_cap;
};

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static int get_workspace(blsh_ctx *ctx, int64_t chunk, bool queue, bool with_m, Workspace *w) {
  const int64_t S = kSlices;
  w->q_cap = queue ? (chunk + 1024 + S - 1) / S + 256 : 0;
  const int64_t stage = ctx->tuning.acc_stage_cap > 0 ? int64_t(ctx->tuning.acc_stage_cap) : kStageDefault;
  w->st_cap = (std::min<int64_t>(chunk, stage) + S - 1) / S;
  const size_t q_bytes = align256(size_t(S) * w->q_cap * 4);
  const size_t st_bytes = align256(size_t(S) * w->st_cap * 4);
  int rc = ensure_workspace(ctx, q_bytes * (with_m ? 2 : 1) + 2 * st_bytes);
  if (rc) return rc;
  w->cnt = ctx->d_slices;
  char *p = static_cast<char *>(ctx->ws);
  w->q_rel = queue ? reinterpret_cast<uint32_t *>(p) : nullptr;
  w->q_m = queue && with_m ? reinterpret_cast<uint32_t *>(p + q_bytes) : nullptr;
  p += q_bytes * (with_m ? 2 : 1);
  w->st_rel = reinterpret_cast<uint32_t *>(p);
  w->st_val = reinterpret_cast<float *>(p + st_bytes);
  return BLSH_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (bayeslsh_verify_noalloc): one
// fixed array per GPU for everything one launch of at most kNaChunk
// candidates needs beyond the caller's inputs and outputs -- the slice
// counters, the decision-table image, the survivor queue (index and m | level
// per entry) and the accepted-pair staging.  A longer call runs as several
// such launches.  Every call on a GPU uses that GPU's copy and leaves its
// contents behind; a call clears the counters it relies on before its first
// launch, so calls that overlap on one GPU race.
//
// In host code `scratch` is a host-side stand-in, not a device address:
// bayeslsh_create looks up each device's address once (hipGetSymbolAddress,
// that device current) and every use goes through that pointer.
// ---------------------------------------------------------------------------
static constexpr size_t align256c(size_t b) { return (b + 255) & ~size_t(255); }
static constexpr int64_t kNaChunk = int64_t(1) << 20;
static constexpr int64_t kNaQueueCap = (kNaChunk + 1024 + kSlices - 1) / kSlices + 256;
static constexpr int64_t kNaStageCap = (kNaChunk + kSlices - 1) / kSlices;
static constexpr size_t kNaCntBytes = align256c(kSliceBufWords * sizeof(int64_t));
static constexpr size_t kNaTabBytes = size_t(40) << 10;   // tables of up to 64 levels of 4096 hashes: 33 KB
static constexpr size_t kNaQBytes = align256c(size_t(kSlices) * kNaQueueCap * 4);
static constexpr size_t kNaStBytes = align256c(size_t(kSlices) * kNaStageCap * 4);
static constexpr size_t kScratchBytes = kNaCntBytes + kNaTabBytes + 2 * kNaQBytes + 2 * kNaStBytes;
static_assert(kScratchBytes <= (size_t(24) << 20), "scratch stays modest");
static_assert((kTabAccOff + size_t(kMaxLevels) * ((64 * kMaxLevels + 1 + 31) / 32)) * 4 <= kNaTabBytes,
              "the largest table image fits its region");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kScratchDevices];

// Address of this file's scratch array on `device` (which must be current);
// looked up once per device.
static int scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return BLSH_OK;   // the allocation-free entry point refuses it
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[device]) return BLSH_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(BLSH_EDEVICE, "scratch address lookup on device %d failed: %s", device, hipGetErrorString(e));
  g_scratch[device] = ptr;
  return BLSH_OK;
}

// The workspace of one launch, carved from the device's scratch array.
static int scratch_workspace(blsh_ctx *ctx, Workspace *w, uint32_t **table) {
  void *base = ctx->device >= 0 && ctx->device < kScratchDevices ? g_scratch[ctx->device] : nullptr;
  if (!base) return fail(BLSH_EDEVICE, "no scratch array on device %d", ctx->device);
  char *p = static_cast<char *>(base);
  w->cnt = reinterpret_cast<int64_t *>(p);
  p += kNaCntBytes;
  *table = reinterpret_cast<uint32_t *>(p);
  p += kNaTabBytes;
  w->q_rel = reinterpret_cast<uint32_t *>(p);
  w->q_m = reinterpret_cast<uint32_t *>(p + kNaQBytes);
  w->q_cap = kNaQueueCap;
  p += 2 * kNaQBytes;
  w->st_rel = reinterpret_cast<uint32_t *>(p);
  w->st_val = reinterpret_cast<float *>(p + kNaStBytes);
  w->st_cap = kNaStageCap;
  return BLSH_OK;
}

static void fill_exact(VerifyArgs &a, const blsh_vectors *v) {
  a.ex_kind = v->kind;
  a.ex_dense = v->dense;
  a.ex_dim = v->dim;
  a.ex_offsets = v->offsets;
  a.ex_indices = v->indices;
  a.ex_values = v->values;
}

// Shared driver of verify / lite / exhaustive.
// Algorithm 1 over BLSH_TILES candidates: launches of at most kTilesChunk
// tiles, each [k_verify_tiles, k_tiles_scan, k_tiles_copy].  The tile kernel
// runs on a persistent grid, each wave with a staging region of its own (no
// atomics; kTilesStage entries in all, each the candidate's absolute index and
// its raw (m, n), so tiles may come in any order of their numbering); the
// running accepted count sits in the context's counter buffer.
static constexpr int64_t kTilesChunk = int64_t(1) << 22;
static constexpr int64_t kTilesStage = int64_t(1) << 27;
static constexpr int64_t kTilesStageLite = int64_t(1) << 27;   // 20 B per entry
// (the tile kernel addresses a launch's descriptors and a wave's staging
// region with 32-bit byte offsets)
static_assert(kTilesChunk * int64_t(sizeof(blsh_tile)) < (int64_t(1) << 31), "descriptor offsets");
static_assert(kTilesStage < (int64_t(1) << 29) && kTilesStageLite < (int64_t(1) << 29), "staging offsets");

static int run_tiles(blsh_ctx *ctx, const blsh_candidates *cand, VerifyArgs a, int k, int n_max, int n_levels,
                     bool intervals, bool lite, hipStream_t s) {
  const int words = (n_levels * k + 1 + 31) / 32;
  int64_t waves = 0;
  int rc = tiles_grid_waves(ctx, k, n_max, intervals, lite, size_t(n_levels) * words * 4, &waves);
  if (rc) return rc;
  // (no more entries than the call has candidates; a wave whose region fills
  // emits directly.  Lite: every position of every tile a wave takes in a
  // launch fits its region, so the launch is sized by the staging.)
  const int64_t stage = ctx->tuning.acc_stage_cap > 0 ? int64_t(ctx->tuning.acc_stage_cap)
                                                      : std::min<int64_t>(lite ? kTilesStageLite : kTilesStage,
                                                                          cand->n_cand);
  int64_t st_cap = std::max<int64_t>(1, stage / waves);   // entries per wave region
  int64_t chunk = ctx->tuning.tiles_per_launch > 0 ? int64_t(ctx->tuning.tiles_per_launch) : kTilesChunk;
  if (lite && ctx->tuning.acc_stage_cap <= 0)   // room for every position of the call's tiles, if it fits
    st_cap = std::min<int64_t>(kTilesStageLite / waves, 256 * ((cand->n_tiles + waves - 1) / waves));
  if (lite) {
    st_cap = std::max<int64_t>(256, st_cap / 256 * 256);
    chunk = std::min<int64_t>(chunk, waves * (st_cap / 256));
  }
  const size_t idx_bytes = align256(size_t(waves) * st_cap * 8), val_bytes = align256(size_t(waves) * st_cap * 4);
  const size_t xy_bytes = lite ? align256(size_t(waves) * st_cap * 8) : 0;
  const size_t cnt_bytes = align256(size_t(waves) * 4), off_bytes = align256(size_t(waves) * 8);
  if ((rc = ensure_workspace(ctx, idx_bytes + val_bytes + xy_bytes + cnt_bytes + off_bytes))) return rc;
  char *p = static_cast<char *>(ctx->ws);
  a.st_idx = reinterpret_cast<uint64_t *>(p);
  a.st_val = reinterpret_cast<float *>(p + idx_bytes);
  a.st_xy = lite ? reinterpret_cast<uint2 *>(p + idx_bytes + val_bytes) : nullptr;
  a.st_cap = st_cap;
  a.wst_cnt = reinterpret_cast<uint32_t *>(p + idx_bytes + val_bytes + xy_bytes);
  int64_t *off = reinterpret_cast<int64_t *>(p + idx_bytes + val_bytes + xy_bytes + cnt_bytes);
  a.tiles = cand->tiles;
  a.n_cand = cand->n_cand;
  {
    const uint64_t bytes = uint64_t(a.n_obj) * uint64_t(a.row_words) * 4u;
    a.sig_buf_bytes = a.n_obj <= (int64_t(1) << 24) && bytes < (uint64_t(1) << 32) ? uint32_t(bytes) : 0u;
  }
  a.c_begin = 0;
  a.pfx = nullptr;
  a.st_raw = lite ? 0 : 1;
  // the running accepted count: the context's counter of staging set 0
  a.acc_total = ctx->d_slices + (size_t(3) * kSlices) * kCntStride;
  if ((rc = launch_zero(ctx, a.acc_total, s))) return fail(rc, "launch failed");
  ctx->slices_dirty = true;   // the single-call paths clear their counters before their next use
  for (int64_t t0 = 0; t0 < cand->n_tiles; t0 += chunk) {
    a.t_begin = t0;
    a.t_end = std::min(cand->n_tiles, t0 + chunk);
    rc = launch_verify_tiles(ctx, a, k, n_max, words, intervals, lite, waves, s);
    if (!rc && lite) rc = launch_tiles_exact(ctx, a, waves, s);
    if (!rc) rc = launch_tiles_flush(ctx, a, waves, off, a.t_end == cand->n_tiles, s);
    if (rc) return rc == BLSH_EDEVICE ? fail(rc, "kernel launch failed: %s", hipGetErrorString(hipGetLastError())) : rc;
  }
  return BLSH_OK;
}

// noalloc: Algorithm 1 only; every buffer beyond the caller's comes from the
// device's scratch array (launches of at most kNaChunk candidates), the table
// image is copied into it, and nothing is allocated.
static int run_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs, const blsh_vectors *exact,
                      double t, double eps, double delta, double gamma, blsh_prior prior, int k, int h,
                      int exhaustive_mode /* -1: early-exit path */, blsh_result *res, void *stream,
                      bool noalloc = false) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  const bool lite = exhaustive_mode == -1 ? (exact != nullptr) : exhaustive_mode == BLSH_REPLAY_LITE;
  const bool tab_lite = lite || exhaustive_mode == BLSH_MLE;  // no concentration bits needed
  int rc = check_params(t, eps, delta, gamma, tab_lite);
  if (rc) return rc;
  int n_max = 0, row_words = 0;
  if ((rc = check_sigs(sigs, k, &n_max, &row_words))) return rc;
  if ((rc = check_prior(sigs->measure, prior))) return rc;
  int64_t n_cand = 0;
  if ((rc = check_cand(cand, &n_cand))) return rc;
  if ((rc = check_result(res))) return rc;
  if (lite) {
    if (h <= 0 || h % k || h > n_max) return fail(BLSH_EINVAL, "Lite: h (%d) must be a positive multiple of k <= n_max", h);
    if ((rc = check_exact(exact, sigs->measure, sigs->n_obj))) return rc;
  }
  const bool exh = exhaustive_mode >= 0;
  if (cand->kind == BLSH_TILES) {
    if (exh || noalloc)
      return fail(BLSH_EINVAL, "BLSH_TILES candidates: bayeslsh_verify and bayeslsh_lite_verify only");
    if (lite && (h % 128 || h > 2048)) return fail(BLSH_EINVAL, "BLSH_TILES candidates, Lite: h must be a multiple of 128 <= 2048");
    if (sigs->measure != BLSH_COSINE) return fail(BLSH_EINVAL, "BLSH_TILES candidates: SRP signatures only");
    if (sigs->layout != BLSH_OBJECT_MAJOR || (uintptr_t(sigs->data) & 15) || row_words % 4)
      return fail(BLSH_EINVAL, "BLSH_TILES candidates: object-major rows of a multiple of 128 hashes, 16-byte aligned");
    if (n_max % 128 || n_max > 2048) return fail(BLSH_EINVAL, "BLSH_TILES candidates: n_max must be a multiple of 128 <= 2048");
  }
  if (exh) {
    if (sigs->measure == BLSH_COSINE) {
      if (sigs->layout != BLSH_OBJECT_MAJOR) return fail(BLSH_EINVAL, "exhaustive: SRP signatures must be OBJECT_MAJOR");
      if (n_max % 128 || n_max > 2048) return fail(BLSH_EINVAL, "exhaustive: SRP n_max must be a multiple of 128 <= 2048");
      if (uintptr_t(sigs->data) & 15 || row_words % 4) return fail(BLSH_EINVAL, "exhaustive: rows must be 16-byte aligned");
    } else if (n_max > 256) {
      return fail(BLSH_EINVAL, "exhaustive: minhash n_max must be <= 256");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n_levels = (lite ? h : n_max) / k;
  TableKey key{int(sigs->measure), t, eps, tab_lite ? 0.0 : delta, tab_lite ? 0.0 : gamma, prior.alpha, prior.beta, k,
               n_levels, tab_lite ? 1 : 0};
  const uint32_t *dtab = nullptr;
  Workspace w{};
  uint32_t *na_table = nullptr;
  std::shared_ptr<HostTable> na_host;
  if (noalloc) {
    if ((rc = scratch_workspace(ctx, &w, &na_table))) return rc;
    if ((rc = get_table(ctx, key, &na_host, nullptr, s))) return rc;
    if (na_host->image.size() * 4 > kNaTabBytes)
      return fail(BLSH_EINVAL, "table of %zu bytes exceeds the %zu-byte scratch region", na_host->image.size() * 4,
                  kNaTabBytes);
    dtab = na_table;
  } else if ((rc = get_table(ctx, key, &na_host, &dtab, s))) {
    return rc;
  }

  VerifyArgs a{};
  fill_cand(a, cand);
  a.sig = sigs->data;
  a.n_obj = sigs->n_obj;
  a.row_words = row_words;
  // first 128 hashes in one 16-byte gather: the caller's prefix array, or
  // object-major rows that a 16-byte load can start
  if (sigs->measure == BLSH_COSINE && sigs->prefix) {
    a.pfx = sigs->prefix;
    a.pfx_stride = 4;
  } else if (sigs->measure == BLSH_COSINE && sigs->layout == BLSH_OBJECT_MAJOR && row_words % 4 == 0 &&
             (uintptr_t(sigs->data) & 15) == 0) {
    a.pfx = sigs->data;
    a.pfx_stride = row_words;
  }
  a.table = dtab;
  a.n_levels = n_levels;
  a.measure = sigs->measure;
  a.code = res->code;
  a.acc_idx = res->acc_idx;
  a.acc_val = res->acc_val;
  a.acc_cap = res->acc_capacity;
  a.n_acc = res->n_accepted;
  a.m_dbg = res->m_debug;
  a.status = ctx->d_status;
  a.mode = exh ? exhaustive_mode : 0;
  a.count_levels = n_max / k;
  a.t = t;
  if (n_cand == 0 || (cand->kind == BLSH_TILES && cand->n_tiles == 0))
    return launch_zero(ctx, res->n_accepted, s) ? fail(BLSH_EDEVICE, "launch failed") : BLSH_OK;
  if (cand->kind == BLSH_TILES) {
    const bool intervals = (na_host->image[kTabFlagOff] & 1u) != 0 && !ctx->tuning.tiles_accept_bitmask;
    if (lite) fill_exact(a, exact);
    // the rows are staged up to the last level: n_max, or h for Lite
    return run_tiles(ctx, cand, a, k, lite ? h : n_max, n_levels, intervals || lite, lite, s);
  }
  // SRP Algorithm 1 with a prefix view: candidates undecided after the first
  // 128 hashes are queued and finished by a second kernel with every lane busy
  const bool tail = !exh && !lite && sigs->measure == BLSH_COSINE && a.pfx != nullptr && 128 / k < n_levels;
  // Lite exact similarities of SRP survivors: with a prefix view the
  // early-exit kernel queues the survivors for k_exact (it then needs no
  // exact-similarity code: fewer registers, no LDS rows, and its waves never
  // wait on one survivor's sparse gathers); otherwise it computes them itself
  const bool fused_exact = lite && exhaustive_mode == -1 && sigs->measure == BLSH_COSINE && a.pfx == nullptr;
  const bool queued = (lite && !fused_exact) || tail;
  // launches are chunked so that no grid exceeds 2^32 work-items (the
  // dispatch's grid size): the comparator runs up to 64 lanes per candidate
  const int64_t chunk = std::min<int64_t>(n_cand, noalloc ? kNaChunk : exh ? kExhChunk : kChunk);
  if (noalloc) {
    // the table image, then every counter of the single-call paths cleared
    // (the array keeps whatever the last call on this GPU left there)
    BLSH_HIP(hipMemcpyAsync(na_table, na_host->image.data(), na_host->image.size() * 4, hipMemcpyHostToDevice, s));
    if ((rc = launch_zero_slices(ctx, w.cnt, s))) return fail(rc, "launch failed");
  } else if ((rc = get_workspace(ctx, chunk, queued, tail, &w))) {
    return rc;
  }
  a.q_rel = w.q_rel;
  a.q_m = w.q_m;
  a.q_cnt = w.cnt + size_t(2) * kSlices * kCntStride;
  a.q_cap = w.q_cap;
  a.st_rel = w.st_rel;
  a.st_val = w.st_val;
  a.st_cap = w.st_cap;
  if (lite) fill_exact(a, exact);
  // the counters of the next set are zero unless an earlier call stopped
  // before its last flush (the allocation-free path cleared its own above and
  // starts from set 0)
  if (!noalloc && ctx->slices_dirty) {
    if ((rc = launch_zero_slices(ctx, w.cnt, s))) return fail(rc, "launch failed");
    ctx->slices_dirty = false;
  }
  int na_set = 0;
  int &set = noalloc ? na_set : ctx->slice_set;
  auto set_cnt = [&](int st) { return w.cnt + size_t(st) * kSlices * kCntStride; };
  auto set_total = [&](int st) { return w.cnt + (size_t(3) * kSlices + st) * kCntStride; };
  for (int64_t c0 = 0; c0 < n_cand; c0 += chunk) {
    a.c_begin = c0;
    a.c_end = std::min(n_cand, c0 + chunk);
    const int cur = set, nxt = cur ^ 1;
    a.acc_cnt = set_cnt(cur);
    a.acc_total = set_total(cur);
    const bool wm = sigs->measure == BLSH_COSINE && sigs->layout == BLSH_WORD_MAJOR;
    if (!noalloc) ctx->slices_dirty = true;
    rc = exh ? launch_exhaustive(ctx, a, k, s) : launch_verify(ctx, a, k, lite, wm, s);
    if (!rc && tail) rc = launch_verify_tail(ctx, a, k, wm, (n_levels * k + 1 + 31) / 32, s);
    if (!rc && queued && !tail) rc = launch_exact(ctx, a, a.c_end - a.c_begin, s);
    if (!rc) rc = launch_acc_flush(ctx, a, set_cnt(nxt), set_total(nxt), a.c_end == n_cand, s);
    if (rc) return rc == BLSH_EDEVICE ? fail(rc, "kernel launch failed: %s", hipGetErrorString(hipGetLastError())) : rc;
    set = nxt;
  }
  if (!noalloc) ctx->slices_dirty = false;
  return BLSH_OK;
}

}  // namespace blsh

using namespace blsh;

extern "C" {

const char *bayeslsh_last_error(void) { return g_err; }
int bayeslsh_version(void) { return BAYESLSH_VERSION; }

int bayeslsh_create(blsh_ctx **out, int device) {
  if (!out) return fail(BLSH_EINVAL, "null output pointer");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(BLSH_EDEVICE, "no HIP device");
  if (device < 0 || device >= n) return fail(BLSH_EINVAL, "device %d out of range", device);
  BLSH_HIP(hipSetDevice(device));
  if (int rc = scratch_init(device)) return rc;
  auto *c = new (std::nothrow) blsh_ctx();
  if (!c) return fail(BLSH_ENOMEM, "host allocation failed");
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  if (hipMalloc(&c->d_status, 256) != hipSuccess) {
    delete c;
    return fail(BLSH_ENOMEM, "status allocation failed");
  }
  if (hipMemset(c->d_status, 0, 256) != hipSuccess) {
    hipFree(c->d_status);
    delete c;
    return fail(BLSH_EDEVICE, "status init failed");
  }
  if (hipMalloc(&c->d_slices, kSliceBufWords * sizeof(int64_t)) != hipSuccess) {
    hipFree(c->d_status);
    delete c;
    return fail(BLSH_ENOMEM, "counter allocation failed");
  }
  if (hipMemset(c->d_slices, 0, kSliceBufWords * sizeof(int64_t)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    hipFree(c->d_slices);
    hipFree(c->d_status);
    delete c;
    return fail(BLSH_EDEVICE, "counter init failed");
  }
  *out = c;
  return BLSH_OK;
}

int bayeslsh_reserve_workspace(blsh_ctx *ctx, size_t bytes, int32_t fixed) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  ctx->ws_fixed = false;
  if (int rc = ensure_workspace(ctx, bytes)) return rc;
  ctx->ws_fixed = fixed != 0;
  return BLSH_OK;
}

int bayeslsh_workspace_bytes(blsh_ctx *ctx, size_t *bytes_host) {
  if (!ctx || !bytes_host) return fail(BLSH_EINVAL, "null argument");
  *bytes_host = ctx->ws_bytes;
  return BLSH_OK;
}

void bayeslsh_destroy(blsh_ctx *ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto &kv : ctx->dev_tables) hipFree(kv.second.ptr);
  for (auto &p : ctx->prof_pending) { hipEventDestroy(p.start); hipEventDestroy(p.stop); }
  if (ctx->batch && ctx->batch_free) ctx->batch_free(ctx->batch);
  if (ctx->ws) hipFree(ctx->ws);
  if (ctx->d_status) hipFree(ctx->d_status);
  if (ctx->d_slices) hipFree(ctx->d_slices);
  if (ctx->tile_buf) hipFree(ctx->tile_buf);
  delete ctx;
}

int bayeslsh_sync(blsh_ctx *ctx, void *stream) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  BLSH_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
  int32_t st = 0;
  BLSH_HIP(hipMemcpy(&st, ctx->d_status, 4, hipMemcpyDeviceToHost));
  if (st != 0) {
    BLSH_HIP(hipMemset(ctx->d_status, 0, 4));
    const char *what = st == BLSH_ETRUNCATED ? "accepted list overflowed acc_capacity"
                       : st == BLSH_EBADID  ? "a candidate referenced an object id >= n_obj"
                       : st == BLSH_EINVAL  ? "invalid input found on the device (empty set)"
                                            : "device error";
    return fail(st, "%s", what);
  }
  return BLSH_OK;
}

int bayeslsh_profile_enable(blsh_ctx *ctx, int enable) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  ctx->prof = enable != 0;
  return BLSH_OK;
}

int bayeslsh_profile_reset(blsh_ctx *ctx) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  for (auto &p : ctx->prof_pending) {
    hipEventSynchronize(p.stop);
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  ctx->prof_pending.clear();
  ctx->prof_acc.clear();
  return BLSH_OK;
}

int bayeslsh_profile_read(blsh_ctx *ctx, const char *name_substr, double *total_ms, int64_t *launches) {
  if (!ctx || !name_substr) return fail(BLSH_EINVAL, "null argument");
  for (auto &p : ctx->prof_pending) {
    BLSH_HIP(hipEventSynchronize(p.stop));
    float ms = 0.f;
    BLSH_HIP(hipEventElapsedTime(&ms, p.start, p.stop));
    auto &acc = ctx->prof_acc[p.name];
    acc.first += ms;
    acc.second += 1;
    hipEventDestroy(p.start);
    hipEventDestroy(p.stop);
  }
  ctx->prof_pending.clear();
  double tot = 0;
  int64_t n = 0;
  for (auto &kv : ctx->prof_acc)
    if (kv.first.find(name_substr) != std::string::npos) { tot += kv.second.first; n += kv.second.second; }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  return BLSH_OK;
}

int bayeslsh_set_tuning(blsh_ctx *ctx, const blsh_tuning *t) {
  if (!ctx || !t) return fail(BLSH_EINVAL, "null argument");
  if (t->gather < 0 || t->gather > 1) return fail(BLSH_EINVAL, "tuning.gather must be 0 or 1");
  if (t->batch_inreg < 0 || t->batch_inreg > kMaxLevels) return fail(BLSH_EINVAL, "tuning.batch_inreg out of range");
  if (t->batch_blocks_per_cu < 0 || t->batch_blocks_per_cu > 32)
    return fail(BLSH_EINVAL, "tuning.batch_blocks_per_cu must be in [0, 32]");
  if (t->batch_spill_cap < 0) return fail(BLSH_EINVAL, "tuning.batch_spill_cap < 0");
  if (t->acc_stage_cap < 0) return fail(BLSH_EINVAL, "tuning.acc_stage_cap < 0");
  if (t->batch_srp_tile != 0 && t->batch_srp_tile != 128 && t->batch_srp_tile != 256 && t->batch_srp_tile != 512)
    return fail(BLSH_EINVAL, "tuning.batch_srp_tile must be 0, 128, 256 or 512");
  if (t->batch_mh_tile != 0 && t->batch_mh_tile != 64 && t->batch_mh_tile != 128)
    return fail(BLSH_EINVAL, "tuning.batch_mh_tile must be 0, 64 or 128");
  if (t->tiles_accept_bitmask < 0 || t->tiles_accept_bitmask > 1)
    return fail(BLSH_EINVAL, "tuning.tiles_accept_bitmask must be 0 or 1");
  if (t->tiles_per_launch < 0 || t->tiles_per_launch > kTilesChunk)
    return fail(BLSH_EINVAL, "tuning.tiles_per_launch must be in [0, 2^22]");
  ctx->tuning.gather = t->gather;
  ctx->tuning.acc_stage_cap = t->acc_stage_cap;
  ctx->tuning.batch_spill_cap = t->batch_spill_cap;
  ctx->tuning.batch_inreg = t->batch_inreg;
  ctx->tuning.batch_blocks_per_cu = t->batch_blocks_per_cu;
  ctx->tuning.batch_srp_tile = t->batch_srp_tile;
  ctx->tuning.batch_mh_tile = t->batch_mh_tile;
  ctx->tuning.tiles_accept_bitmask = t->tiles_accept_bitmask;
  ctx->tuning.tiles_per_launch = t->tiles_per_launch;
  return BLSH_OK;
}

int bayeslsh_get_tuning(blsh_ctx *ctx, blsh_tuning *t) {
  if (!ctx || !t) return fail(BLSH_EINVAL, "null argument");
  *t = ctx->tuning;
  return BLSH_OK;
}

int bayeslsh_posterior_table(blsh_ctx *ctx, blsh_measure measure, double t, double epsilon, double delta,
                             double gamma, blsh_prior prior, int32_t k, int32_t n_levels, int32_t lite,
                             int32_t *min_matches_host, uint32_t *accept_host, double *min_margin_host) {
  int rc = check_params(t, epsilon, delta, gamma, lite != 0);
  if (rc) return rc;
  if (measure != BLSH_JACCARD && measure != BLSH_COSINE) return fail(BLSH_EINVAL, "bad measure");
  if ((rc = check_prior(measure, prior))) return rc;
  if (k <= 0 || k > 4096 || n_levels <= 0 || n_levels > kMaxLevels) return fail(BLSH_EINVAL, "bad k or n_levels");
  TableKey key{int(measure), t, epsilon, lite ? 0.0 : delta, lite ? 0.0 : gamma, prior.alpha, prior.beta, k,
               n_levels, lite ? 1 : 0};
  std::shared_ptr<HostTable> ht;
  if (ctx) {
    if ((rc = get_table(ctx, key, &ht, nullptr, nullptr))) return rc;
  } else {  // no context (e.g. a host without a GPU): build without caching
    ht = std::make_shared<HostTable>();
    if ((rc = build_table(key, ht.get()))) return rc;
  }
  if (min_matches_host) std::memcpy(min_matches_host, ht->min_matches.data(), 4 * ht->min_matches.size());
  if (accept_host) std::memcpy(accept_host, ht->accept.data(), 4 * ht->accept.size());
  if (min_margin_host) *min_margin_host = ht->min_margin;
  return BLSH_OK;
}

int bayeslsh_minhash_sigs(blsh_ctx *ctx, const blsh_vectors *sets, const uint32_t *a, const uint32_t *b,
                          int32_t n_hashes, uint32_t *sigs_out, void *stream) {
  if (!ctx || !sets || !a || !b || !sigs_out) return fail(BLSH_EINVAL, "null argument");
  if (sets->kind != BLSH_SETS || !sets->offsets || !sets->indices) return fail(BLSH_EINVAL, "minhash needs SETS vectors");
  if (n_hashes <= 0 || n_hashes > 1024) return fail(BLSH_EINVAL, "n_hashes must be in [1, 1024]");
  if (sets->n_obj <= 0) return BLSH_OK;
  return launch_minhash(ctx, sets->offsets, sets->indices, sets->n_obj, a, b, n_hashes, sigs_out,
                        static_cast<hipStream_t>(stream));
}

int bayeslsh_srp_sigs(blsh_ctx *ctx, const blsh_vectors *vecs, const float *planes, int32_t n_bits, uint64_t seed,
                      blsh_layout layout, int32_t flags, uint32_t *bits_out, void *stream) {
  if (!ctx || !vecs || !bits_out) return fail(BLSH_EINVAL, "null argument");
  if (flags & ~int32_t(BLSH_SRP_PLANES_Q16)) return fail(BLSH_EINVAL, "unknown SRP flags 0x%x", unsigned(flags));
  const bool q16 = (flags & BLSH_SRP_PLANES_Q16) != 0;
  if (n_bits <= 0 || n_bits % 32) return fail(BLSH_EINVAL, "n_bits must be a positive multiple of 32");
  if (layout != BLSH_OBJECT_MAJOR && layout != BLSH_WORD_MAJOR) return fail(BLSH_EINVAL, "bad layout");
  if (vecs->n_obj <= 0) return BLSH_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (vecs->kind == BLSH_DENSE) {
    if (!vecs->dense || !planes) return fail(BLSH_EINVAL, "dense SRP needs vectors and planes");
    if (uintptr_t(vecs->dense) & 15) return fail(BLSH_EINVAL, "dense vectors must be 16-byte aligned");
    if (q16) return fail(BLSH_EINVAL, "BLSH_SRP_PLANES_Q16 applies to generated (CSR) planes only");
    return launch_srp_dense(ctx, vecs->dense, vecs->n_obj, vecs->dim, planes, n_bits, layout == BLSH_WORD_MAJOR,
                            bits_out, s);
  }
  if (vecs->kind == BLSH_CSR) {
    if (!vecs->offsets || !vecs->indices || !vecs->values) return fail(BLSH_EINVAL, "CSR SRP needs offsets/indices/values");
    if (planes) return fail(BLSH_EINVAL, "CSR SRP generates its planes: pass planes = NULL");
    if (n_bits > 2048) return fail(BLSH_EINVAL, "CSR SRP: n_bits must be <= 2048");
    return launch_srp_sparse(ctx, vecs->offsets, vecs->indices, vecs->values, vecs->n_obj, vecs->dim, n_bits, seed,
                             layout == BLSH_WORD_MAJOR, q16, bits_out, s);
  }
  return fail(BLSH_EINVAL, "SRP needs DENSE or CSR vectors");
}

int bayeslsh_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs, double t, double epsilon,
                    double delta, double gamma, blsh_prior prior, int32_t k, blsh_result *res, void *stream) {
  return run_verify(ctx, cand, sigs, nullptr, t, epsilon, delta, gamma, prior, k, 0, -1, res, stream);
}

int bayeslsh_verify_noalloc(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs, double t,
                            double epsilon, double delta, double gamma, blsh_prior prior, int32_t k,
                            blsh_result *res, void *stream) {
  if (ctx && (ctx->device < 0 || ctx->device >= kScratchDevices))
    return fail(BLSH_EINVAL, "bayeslsh_verify_noalloc: device %d has no scratch array (devices 0..%d)", ctx->device,
                kScratchDevices - 1);
  return run_verify(ctx, cand, sigs, nullptr, t, epsilon, delta, gamma, prior, k, 0, -1, res, stream, true);
}

int bayeslsh_lite_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs, const blsh_vectors *exact,
                         double t, double epsilon, blsh_prior prior, int32_t h, int32_t k, blsh_result *res,
                         void *stream) {
  if (!exact) return fail(BLSH_EINVAL, "Lite needs exact vectors");
  return run_verify(ctx, cand, sigs, exact, t, epsilon, 0.5, 0.5, prior, k, h, -1, res, stream);
}

static int batched_common(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand,
                          int64_t n_cand, const blsh_sigs *jac, const blsh_sigs *cos, double epsilon, double delta,
                          double gamma, blsh_prior prior, int32_t kj, int32_t kc, int32_t *k_used, blsh_result *res,
                          void *stream, int mode) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  int rc = check_params(0.5, epsilon, delta, gamma, false);
  if (rc) return rc;
  for (int32_t k : {kj, kc})
    if (k != 0 && k != 16 && k != 32 && k != 64) return fail(BLSH_EINVAL, "k must be 0 (autotune), 16, 32 or 64");
  if (n_lists < 0 || n_cand < 0 || n_cand > (int64_t(1) << 40)) return fail(BLSH_EINVAL, "bad list or candidate count");
  if (n_lists > 0 && !lists) return fail(BLSH_EINVAL, "null list descriptors");
  if (n_cand > 0 && !cand) return fail(BLSH_EINVAL, "null candidates");
  if ((rc = check_result(res))) return rc;
  if ((rc = check_prior(BLSH_JACCARD, prior))) return rc;
  for (int64_t i = 0; i < n_lists; ++i) {
    const blsh_list_desc &d = lists[i];
    if (d.measure != BLSH_JACCARD && d.measure != BLSH_COSINE) return fail(BLSH_EINVAL, "list %lld: bad measure", (long long)i);
    if (!in01(d.t)) return fail(BLSH_EINVAL, "list %lld: t must be in (0,1)", (long long)i);
    if (d.offset < 0 || d.length < 0 || d.offset + d.length > n_cand)
      return fail(BLSH_EINVAL, "list %lld: range outside [0, n_cand)", (long long)i);
    if (mode == 1 && (d.measure == BLSH_JACCARD ? kj : kc) == 0)
      return fail(BLSH_EINVAL, "the exhaustive comparator needs an explicit k for every measure it runs");
  }
  if (mode == 1) {
    for (const blsh_sigs *sg : {jac, cos}) {
      if (!sg) continue;
      int nm = 0, rw = 0;
      const int32_t k = sg->measure == BLSH_JACCARD ? kj : kc;
      if (k == 0) continue;   // no list of this measure (checked above)
      if ((rc = check_sigs(sg, k, &nm, &rw))) return rc;
      if (sg->layout != BLSH_OBJECT_MAJOR || (uintptr_t(sg->data) & 15) || rw % 4)
        return fail(BLSH_EINVAL, "exhaustive: object-major, 16-byte aligned rows required");
      if (sg->measure == BLSH_COSINE && nm != 128 && nm != 256 && nm != 512 && nm != 1024 && nm != 2048)
        return fail(BLSH_EINVAL, "exhaustive: SRP n_max must be 128, 256, 512, 1024 or 2048");
      if (sg->measure == BLSH_JACCARD && nm % 64)
        return fail(BLSH_EINVAL, "exhaustive: minhash n_max must be a multiple of 64");
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_lists == 0 || n_cand == 0) {
    if (launch_zero(ctx, res->n_accepted, s)) return fail(BLSH_EDEVICE, "launch failed");
    if (k_used) { k_used[0] = kj; k_used[1] = kc; }
    return BLSH_OK;
  }
  return verify_batched(ctx, lists, n_lists, cand, n_cand, jac, cos, epsilon, delta, gamma, prior, kj, kc, res, k_used,
                        s, check_sigs, mode);
}

int bayeslsh_verify_batched(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand,
                            int64_t n_cand, const blsh_sigs *jac, const blsh_sigs *cos, double epsilon, double delta,
                            double gamma, blsh_prior prior, int32_t kj, int32_t kc, int32_t *k_used,
                            blsh_result *res, void *stream) {
  return batched_common(ctx, lists, n_lists, cand, n_cand, jac, cos, epsilon, delta, gamma, prior, kj, kc, k_used, res,
                        stream, 0);
}

int bayeslsh_exhaustive_batched(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand,
                                int64_t n_cand, const blsh_sigs *jac, const blsh_sigs *cos, double epsilon,
                                double delta, double gamma, blsh_prior prior, int32_t kj, int32_t kc,
                                blsh_result *res, void *stream) {
  return batched_common(ctx, lists, n_lists, cand, n_cand, jac, cos, epsilon, delta, gamma, prior, kj, kc, nullptr,
                        res, stream, 1);
}

int bayeslsh_exact_similarity(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_vectors *vecs,
                              double *sim_out, void *stream) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  int64_t n_cand = 0;
  int rc = check_cand(cand, &n_cand);
  if (rc) return rc;
  if (!vecs) return fail(BLSH_EINVAL, "exact vectors: null");
  if ((rc = check_exact(vecs, vecs->kind == BLSH_SETS ? BLSH_JACCARD : BLSH_COSINE, 0))) return rc;
  if (vecs->n_obj <= 0 || vecs->n_obj > 0xFFFFFFFFll) return fail(BLSH_EINVAL, "exact vectors: n_obj out of range");
  if (n_cand > 0 && !sim_out) return fail(BLSH_EINVAL, "sim_out: null");
  VerifyArgs a{};
  fill_cand(a, cand);
  fill_exact(a, vecs);
  a.n_obj = vecs->n_obj;
  a.status = ctx->d_status;
  a.c_begin = 0;
  a.c_end = n_cand;
  return launch_exact_pairs(ctx, a, sim_out, static_cast<hipStream_t>(stream)) ? fail(BLSH_EDEVICE, "launch failed")
                                                                                : BLSH_OK;
}

int bayeslsh_band_candidates(blsh_ctx *ctx, const blsh_sigs *band_sigs, int32_t n_bands, int32_t band_bits,
                             int32_t max_bucket, int32_t order_tile, uint32_t *x_out, uint32_t *y_out,
                             int64_t capacity, int64_t *n_pairs_host, void *stream) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  if (!n_pairs_host) return fail(BLSH_EINVAL, "n_pairs_host: null");
  *n_pairs_host = 0;
  const blsh_sigs *g = band_sigs;
  if (!g || !g->data) return fail(BLSH_EINVAL, "band signatures: null");
  if (g->measure != BLSH_COSINE) return fail(BLSH_EINVAL, "banding takes sign-random-projection bits");
  if (g->layout != BLSH_OBJECT_MAJOR && g->layout != BLSH_WORD_MAJOR) return fail(BLSH_EINVAL, "bad layout");
  if (g->n_obj <= 0 || g->n_obj > 0xFFFFFFFFll) return fail(BLSH_EINVAL, "band signatures: n_obj out of range");
  if (g->n_hashes <= 0 || g->n_hashes % 32) return fail(BLSH_EINVAL, "band signatures: n_hashes must be a multiple of 32");
  if (band_bits < 1 || band_bits > 32 || n_bands < 1 || n_bands > 64)
    return fail(BLSH_EINVAL, "banding: 1 <= band_bits <= 32 and 1 <= n_bands <= 64");
  if (int64_t(n_bands) * band_bits > g->n_hashes)
    return fail(BLSH_EINVAL, "banding: n_bands * band_bits (%d) > n_hashes (%d)", n_bands * band_bits, g->n_hashes);
  if (max_bucket < 0 || capacity < 0) return fail(BLSH_EINVAL, "banding: negative max_bucket or capacity");
  if (order_tile != 0 && order_tile != 16) return fail(BLSH_EINVAL, "banding: order_tile must be 0 or 16");
  if (capacity > 0 && (!x_out || !y_out)) return fail(BLSH_EINVAL, "banding: null outputs");
  return band_candidates(ctx, g->data, g->n_obj, g->n_hashes / 32, g->layout == BLSH_WORD_MAJOR, n_bands, band_bits,
                         max_bucket, order_tile, x_out, y_out, capacity, n_pairs_host,
                         static_cast<hipStream_t>(stream), nullptr);
}

int bayeslsh_band_tiles(blsh_ctx *ctx, const blsh_sigs *band_sigs, int32_t n_bands, int32_t band_bits,
                        int32_t max_bucket, blsh_tile *tiles_out, int64_t tiles_capacity, int64_t *n_tiles_host,
                        int64_t *n_pairs_host, void *stream) {
  if (!ctx) return fail(BLSH_EINVAL, "null context");
  if (!n_pairs_host || !n_tiles_host) return fail(BLSH_EINVAL, "n_tiles_host / n_pairs_host: null");
  *n_pairs_host = 0;
  *n_tiles_host = 0;
  const blsh_sigs *g = band_sigs;
  if (!g || !g->data) return fail(BLSH_EINVAL, "band signatures: null");
  if (g->measure != BLSH_COSINE) return fail(BLSH_EINVAL, "banding takes sign-random-projection bits");
  if (g->layout != BLSH_OBJECT_MAJOR && g->layout != BLSH_WORD_MAJOR) return fail(BLSH_EINVAL, "bad layout");
  if (g->n_obj <= 0 || g->n_obj > 0xFFFFFFFFll) return fail(BLSH_EINVAL, "band signatures: n_obj out of range");
  if (g->n_hashes <= 0 || g->n_hashes % 32) return fail(BLSH_EINVAL, "band signatures: n_hashes must be a multiple of 32");
  if (band_bits < 1 || band_bits > 32 || n_bands < 1 || n_bands > 64)
    return fail(BLSH_EINVAL, "banding: 1 <= band_bits <= 32 and 1 <= n_bands <= 64");
  if (int64_t(n_bands) * band_bits > g->n_hashes)
    return fail(BLSH_EINVAL, "banding: n_bands * band_bits (%d) > n_hashes (%d)", n_bands * band_bits, g->n_hashes);
  if (max_bucket < 0 || tiles_capacity < 0) return fail(BLSH_EINVAL, "banding: negative max_bucket or capacity");
  if (tiles_capacity > 0 && !tiles_out) return fail(BLSH_EINVAL, "banding tiles: null tiles_out");
  if (uintptr_t(tiles_out) & 15) return fail(BLSH_EINVAL, "banding tiles: tiles_out must be 16-byte aligned");
  BandTilesOut to{tiles_out, tiles_capacity, n_tiles_host};
  return band_candidates(ctx, g->data, g->n_obj, g->n_hashes / 32, g->layout == BLSH_WORD_MAJOR, n_bands, band_bits,
                         max_bucket, 16, nullptr, nullptr, 0, n_pairs_host, static_cast<hipStream_t>(stream), &to);
}

int bayeslsh_fit_prior(const double *sim_host, int64_t r, blsh_prior *prior_out, int32_t *uniform_host) {
  if (!prior_out) return fail(BLSH_EINVAL, "prior_out: null");
  if (r < 0 || (r > 0 && !sim_host)) return fail(BLSH_EINVAL, "bad sample");
  // Section 4.1, method of moments: sample mean and (population) variance
  double mean = 0.0;
  for (int64_t i = 0; i < r; ++i) {
    if (!(sim_host[i] >= 0.0 && sim_host[i] <= 1.0)) return fail(BLSH_EINVAL, "similarity %lld outside [0,1]", (long long)i);
    mean += sim_host[i];
  }
  bool uniform = r < 2;
  double alpha = 1.0, beta = 1.0;
  if (!uniform) {
    mean /= double(r);
    double var = 0.0;
    for (int64_t i = 0; i < r; ++i) var += (sim_host[i] - mean) * (sim_host[i] - mean);
    var /= double(r);
    const double spread = mean * (1.0 - mean);
    // no Beta has these moments (or only one with parameters past the table
    // builder's range): keep the uniform prior
    if (!(var > 0.0) || !(var < spread)) {
      uniform = true;
    } else {
      const double common = spread / var - 1.0;
      alpha = mean * common;
      beta = (1.0 - mean) * common;
      if (!(alpha > 0.0 && beta > 0.0 && alpha <= 1e6 && beta <= 1e6)) {
        uniform = true;
        alpha = beta = 1.0;
      }
    }
  }
  prior_out->alpha = alpha;
  prior_out->beta = beta;
  if (uniform_host) *uniform_host = uniform ? 1 : 0;
  return BLSH_OK;
}

int bayeslsh_exhaustive_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs,
                               const blsh_vectors *exact, double t, double epsilon, double delta, double gamma,
                               blsh_prior prior, int32_t k, int32_t h, blsh_exhaustive_mode mode, blsh_result *res,
                               void *stream) {
  if (mode != BLSH_REPLAY && mode != BLSH_REPLAY_LITE && mode != BLSH_MLE) return fail(BLSH_EINVAL, "bad mode");
  if (mode == BLSH_MLE) { delta = 0.5; gamma = 0.5; }
  return run_verify(ctx, cand, sigs, mode == BLSH_REPLAY_LITE ? exact : nullptr, t, epsilon, delta, gamma, prior, k,
                    h, int(mode), res, stream);
}

}  // extern "C"
