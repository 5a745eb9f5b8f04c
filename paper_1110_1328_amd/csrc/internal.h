// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/bayeslsh.h"

namespace blsh {

constexpr int kMaxLevels = 64;

// Thread-local error message; returns `code` for convenient `return fail(...)`.
int fail(int code, const char *fmt, ...);

#define BLSH_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::blsh::fail(BLSH_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Posterior decision table (Section 4.3): per level j, n = (j+1) k.
// ---------------------------------------------------------------------------
struct TableKey {
  int measure;
  double t, epsilon, delta, gamma, alpha, beta;
  int k, n_levels, lite;
  bool operator<(const TableKey &o) const {
    return std::tie(measure, t, epsilon, delta, gamma, alpha, beta, k, n_levels, lite) <
           std::tie(o.measure, o.t, o.epsilon, o.delta, o.gamma, o.alpha, o.beta, o.k, o.n_levels, o.lite);
  }
};

struct HostTable {
  int k = 0, n_levels = 0, n_max = 0, words = 0;
  std::vector<int32_t> min_matches;   // [n_levels]
  std::vector<uint32_t> accept;       // [n_levels][words]
  // smallest |probability - threshold| over every evaluated test, and where
  // (n, m, kind: 0 prune, 1 concentration)
  double min_margin = 1.0;
  int margin_n = 0, margin_m = 0, margin_kind = 0;
  std::vector<uint32_t> image;        // the device image (layout below), built once
};

// A table whose smallest margin is below this is refused (BLSH_EINVAL): the
// host quadrature, the binomial sums and any other correct evaluation agree
// far more closely than this, so above it every decision is unique.
constexpr double kTieMargin = 1e-9;

// Device image of a table, read by every verify kernel into LDS.
// Layout of the device buffer (32-bit words):
//   [0] k  [1] n_levels  [2] words  [3] measure
//   [4..5] alpha (double)  [6..7] beta (double)  [8..9] t (double)
//   [10] flags: bit 0 set when every level's accept set, restricted to
//        m >= min_matches, is an interval [min_accept, n] (or empty)
//   [16 .. 16+64)        min_matches
//   [80 .. 80+64)        min_accept (n+1 when nothing is accepted; meaningful
//                        when flag bit 0 is set)
//   [144 .. 144+L*words) accept bits
constexpr int kTabFlagOff = 10;
constexpr int kTabMinOff = 16;
constexpr int kTabAloOff = 16 + kMaxLevels;
constexpr int kTabAccOff = 16 + 2 * kMaxLevels;

int build_table(const TableKey &key, HostTable *out);  // host FP64, tables.cpp

struct DevTable {
  uint32_t *ptr = nullptr;
  size_t words = 0;
};

struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
};

}  // namespace blsh

struct blsh_ctx {
  int device = 0;
  int n_cu = 256;
  std::mutex mu;
  std::map<blsh::TableKey, std::shared_ptr<blsh::HostTable>> host_tables;
  std::map<blsh::TableKey, blsh::DevTable> dev_tables;
  // device status word: first error raised by a kernel (0 = none)
  int32_t *d_status = nullptr;
  // counters of the single-call verification paths: two sets of staging
  // slice counts (launches alternate between them; slice_set names the next
  // one, whose counts and running count are zero between calls), the queue
  // slice counts, the two running accepted counts; slices_dirty: a call
  // stopped before its last flush
  int64_t *d_slices = nullptr;
  int slice_set = 0;
  bool slices_dirty = false;
  // survivor workspace
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_fixed = false;   // set by bayeslsh_reserve_workspace: calls never grow ws
  // banding: per-tile counts and offsets of the tiled emission order
  void *tile_buf = nullptr;
  size_t tile_bytes = 0;
  // tuning (bayeslsh_set_tuning; last_* fields report the last batched call)
  blsh_tuning tuning{};
  // batched-call state (persistent buffers, captured graphs, autotune cache)
  void *batch = nullptr;
  void (*batch_free)(void *) = nullptr;
  // profiling
  bool prof = false;
  std::vector<blsh::ProfRec> prof_pending;
  std::map<std::string, std::pair<double, int64_t>> prof_acc;
};

namespace blsh {
int get_table(blsh_ctx *ctx, const TableKey &key, std::shared_ptr<HostTable> *host, const uint32_t **dev,
              hipStream_t stream);
int ensure_workspace(blsh_ctx *ctx, size_t bytes);

// Tiles output of the banding (bayeslsh_band_tiles): the tile descriptors of
// all bands.
struct BandTilesOut {
  blsh_tile *tiles;
  int64_t tile_cap;
  int64_t *n_tiles;   // host
};

// Device-to-device copy of one request's candidate ids into the serving arena
// (ids src[0, n) to arena[dst, dst + n)).
struct CopyJob {
  const uint32_t *src;
  int64_t dst;
  int64_t n;
};
constexpr int kCopyJobs = 64;
// Enqueue the copies jobs[0, n_jobs) (n_jobs <= kCopyJobs) as one launch.
int gather_copy(const CopyJob *jobs, int n_jobs, uint32_t *arena, hipStream_t s);
// Radix sort of n (position, value) pairs by the low key_bits bits of the
// position.  tmp == nullptr: only sets *tmp_bytes (rocPRIM's convention).
int sort_accepted(const uint64_t *key_in, const float *val_in, uint64_t *key_out, float *val_out, int64_t n,
                  int key_bits, void *tmp, size_t *tmp_bytes, hipStream_t s);

// Launch helper with optional event bracketing.
struct LaunchScope {
  blsh_ctx *ctx;
  hipStream_t stream;
  const char *name;
  hipEvent_t a{}, b{};
  bool on;
  LaunchScope(blsh_ctx *c, hipStream_t s, const char *n);
  ~LaunchScope();
};
}  // namespace blsh
