// LSH banding candidate generation (Section 2): the hashes of an object are
// cut into n_bands bands of band_bits sign-random-projection bits each, and
// objects whose band key is equal in some band become a candidate pair.  A
// pair is emitted once, in the first band where its two keys are equal.
//
// Per band, on the device:
//   keys      every object's key of every band (band-major for the sort,
//             object-major for the first-band test), from the packed bits;
//   sort      (key, id) pairs by key, stable (rocPRIM radix sort), so each
//             bucket lists its members by increasing id;
//   bounds    the bucket [start, end) of every sorted position;
//   count     one wave per member row p: partners q in (p, end), kept when no
//             earlier band has equal keys -> kept pairs per row;
//   scan      exclusive prefix of the row counts (rocPRIM) -> output offsets;
//   emit      the same walk writes (x, y) = (ids[p], ids[q]) at the row's
//             offset plus the lane's ballot rank, so the output order is band
//             by band, bucket by increasing key, row by increasing id, partner
//             by increasing id (x < y).
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "device_common.h"

namespace blsh {

constexpr int kBandBlock = 256;

// Key of band j of object i: bits [j b, j b + b) of its signature (LSB-first).
__global__ __launch_bounds__(kBandBlock) void k_band_keys(const uint32_t *sig, int64_t n_obj, int32_t row_words,
                                                          int32_t word_major, int32_t n_bands, int32_t band_bits,
                                                          uint32_t *keys_bm, uint32_t *keys_om) {
  const int64_t i = int64_t(blockIdx.x) * kBandBlock + threadIdx.x;
  if (i >= n_obj) return;
  const uint32_t mask = band_bits == 32 ? 0xFFFFFFFFu : ((1u << band_bits) - 1u);
  auto word = [&](int w) -> uint32_t {
    return word_major ? sig[size_t(w) * n_obj + i] : sig[size_t(i) * row_words + w];
  };
  for (int j = 0; j < n_bands; ++j) {
    const int o = j * band_bits, w = o >> 5, sh = o & 31;
    uint32_t v = word(w) >> sh;
    if (sh + band_bits > 32) v |= word(w + 1) << (32 - sh);
    v &= mask;
    keys_bm[size_t(j) * n_obj + i] = v;
    keys_om[size_t(i) * n_bands + j] = v;
  }
}

__global__ void k_iota(uint32_t *ids, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) ids[i] = uint32_t(i);
}

// [start, end) of the bucket of every sorted position (the thread at a bucket
// start walks its bucket).
__global__ __launch_bounds__(kBandBlock) void k_bucket_bounds(const uint32_t *skeys, int64_t n, uint32_t *bstart,
                                                              uint32_t *bend) {
  const int64_t p = int64_t(blockIdx.x) * kBandBlock + threadIdx.x;
  if (p >= n || (p > 0 && skeys[p] == skeys[p - 1])) return;
  int64_t e = p + 1;
  while (e < n && skeys[e] == skeys[p]) ++e;
  for (int64_t q = p; q < e; ++q) {
    bstart[q] = uint32_t(p);
    bend[q] = uint32_t(e);
  }
}

struct BandArgs {
  const uint32_t *sids;      // sorted ids of this band
  const uint32_t *bstart, *bend;
  const uint32_t *keys_om;   // [n_obj][n_bands]
  int64_t n_obj;
  int32_t n_bands, band;
  int32_t max_bucket;        // 0: every member; else the first max_bucket members of a bucket
  int64_t *row_count;        // count pass
  const int64_t *row_off;    // emit pass
  const int64_t *base;       // emit pass: output offset of this band
  uint32_t *x_out, *y_out;
  int64_t capacity;
};

// One wave per member row p.  EMIT = false counts the kept pairs of the row;
// EMIT = true writes them in order.
template <bool EMIT>
__global__ __launch_bounds__(kBandBlock) void k_band_pairs(BandArgs a) {
  const int lane = lane_id();
  const int64_t waves = int64_t(gridDim.x) * (kBandBlock / kWave);
  const int64_t w0 = int64_t(blockIdx.x) * (kBandBlock / kWave) +
                     int64_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave));
  const int64_t out0 = EMIT ? *a.base : 0;
  for (int64_t p = w0; p < a.n_obj; p += waves) {
    const int64_t s = a.bstart[p];
    int64_t e = a.bend[p];
    int64_t kept = 0;
    if (a.max_bucket > 0) e = min<int64_t>(e, s + a.max_bucket);
    if (p + 1 < e) {
      const uint32_t x = a.sids[p];
      const uint32_t *kx = a.keys_om + size_t(x) * a.n_bands;
      const int64_t off = EMIT ? out0 + a.row_off[p] : 0;
      for (int64_t q0 = p + 1; q0 < e; q0 += kWave) {
        const int64_t q = q0 + lane;
        bool keep = false;
        uint32_t y = 0;
        if (q < e) {
          y = a.sids[q];
          const uint32_t *ky = a.keys_om + size_t(y) * a.n_bands;
          keep = true;
          for (int j = 0; j < a.band; ++j)   // collided in an earlier band: emitted there
            if (kx[j] == ky[j]) { keep = false; break; }
        }
        const uint64_t mask = __ballot(keep);
        if (EMIT && keep) {
          const int64_t pos = off + kept + int64_t(lanes_below(mask));
          if (pos < a.capacity) {
            a.x_out[pos] = x;
            a.y_out[pos] = y;
          }
        }
        kept += __popcll(mask);
      }
    }
    if (!EMIT && lane == 0) a.row_count[p] = kept;
  }
}

// ---------------------------------------------------------------------------
// Tiled emission order: the upper triangle of a bucket's member positions cut
// into kTile x kTile tiles, listed by tile row, then tile column, each tile
// row-major -- a run of 256 candidates then touches about 2 kTile objects
// instead of one row's ~256, which the verification kernels' L1 reuses.
// ---------------------------------------------------------------------------
constexpr int kTile = 16;   // 16 x 16 = 256 pair positions: one wave, 4 per lane

// flag[p] = 1 where p starts a bucket
__global__ __launch_bounds__(kBandBlock) void k_start_flags(const uint32_t *bstart, int64_t n, uint32_t *flag) {
  const int64_t p = int64_t(blockIdx.x) * kBandBlock + threadIdx.x;
  if (p < n) flag[p] = bstart[p] == uint32_t(p) ? 1u : 0u;
}

// meta[0] = number of buckets (after the exclusive scan of the flags)
__global__ void k_count_buckets(const uint32_t *flag, const uint32_t *bidx, int64_t n, int64_t *meta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) meta[0] = n > 0 ? int64_t(bidx[n - 1]) + flag[n - 1] : 0;
}

// Bucket b (starting at position p): its start, its member count (capped at
// max_bucket) and its number of tiles nT (nT + 1) / 2, nT = ceil(len / kTile).
__global__ __launch_bounds__(kBandBlock) void k_bucket_tiles(const uint32_t *bstart, const uint32_t *bend,
                                                             const uint32_t *bidx, int64_t n, int32_t max_bucket,
                                                             uint32_t *bpos, uint32_t *blen, int64_t *ntile) {
  const int64_t p = int64_t(blockIdx.x) * kBandBlock + threadIdx.x;
  if (p >= n || bstart[p] != uint32_t(p)) return;
  const uint32_t b = bidx[p];
  uint32_t len = bend[p] - uint32_t(p);
  if (max_bucket > 0) len = min(len, uint32_t(max_bucket));
  bpos[b] = uint32_t(p);
  blen[b] = len;
  const int64_t nt = len >= 2 ? (int64_t(len) + kTile - 1) / kTile : 0;
  ntile[b] = nt * (nt + 1) / 2;
}

// meta[1] = number of tiles of the band
__global__ void k_count_tiles(const int64_t *toff, const int64_t *ntile, int64_t nb, int64_t *meta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) meta[1] = nb > 0 ? toff[nb - 1] + ntile[nb - 1] : 0;
}

struct TileArgs {
  const uint32_t *sids;      // sorted ids of this band
  const uint32_t *keys_om;   // [n_obj][n_bands]
  int32_t n_bands, band;
  const uint32_t *bpos, *blen;
  const int64_t *toff;       // first tile of each bucket
  int64_t n_buckets, n_tiles;
  int64_t *tcnt;             // count pass: kept pairs per tile
  uint64_t *tmask;           // count pass writes, emit pass reads: the tile's 4 keep ballots
  const int64_t *tcoff;      // emit pass: their exclusive prefix
  const int64_t *base;       // emit pass: output offset of this band
  uint32_t *x_out, *y_out;
  int64_t capacity;
};

struct TileAt {
  int64_t len, p0, ar, tb;
  bool ok;
};

// Tile t of the band: its bucket (the last b with toff[b] <= t), the bucket's
// length and first sorted position, the tile's column index tb and the
// lane's row ar (tile (ta, tb), tb >= ta: rows before ta hold
// S(ta) = ta nt - ta (ta - 1) / 2 tiles).  ok = false past the last tile.
__device__ inline TileAt tile_at(const TileArgs &a, int64_t t, int lane) {
  TileAt r{0, 0, 0, 0, t < a.n_tiles};
  if (!r.ok) return r;
  int64_t lo = 0, hi = a.n_buckets - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (a.toff[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int64_t lt = t - a.toff[lo];
  r.len = a.blen[lo];
  const int64_t nt = (r.len + kTile - 1) / kTile;
  auto S = [nt](int64_t q) { return q * nt - q * (q - 1) / 2; };
  const double q2 = double(2 * nt + 1);
  int64_t ta = int64_t((q2 - sqrt(max(0.0, q2 * q2 - 8.0 * double(lt)))) / 2.0);
  ta = max<int64_t>(0, min(ta, nt - 1));
  while (ta > 0 && S(ta) > lt) --ta;
  while (ta + 1 < nt && S(ta + 1) <= lt) ++ta;
  r.tb = ta + (lt - S(ta));
  r.p0 = a.bpos[lo];
  r.ar = ta * kTile + (4 * lane) / kTile;
  return r;
}

// One wave per tile: lane l holds the tile's pair positions 4l .. 4l + 3
// (row-major), so lanes, then a lane's four slots, are in output order.  The
// count pass runs the earlier-band test and keeps its four ballots per tile;
// the emit pass reads them back instead of testing again.
template <bool EMIT>
__global__ __launch_bounds__(kBandBlock) void k_band_tiles(TileArgs a) {
  const int lane = lane_id();
  const int64_t waves = int64_t(gridDim.x) * (kBandBlock / kWave);
  const int64_t w0 = int64_t(blockIdx.x) * (kBandBlock / kWave) +
                     int64_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave));
  const int64_t out0 = EMIT ? *a.base : 0;
  for (int64_t t = w0; t < a.n_tiles; t += waves) {
    const TileAt T = tile_at(a, t, lane);
    const int64_t len = T.len, tb = T.tb, p0 = T.p0;
    const int64_t ar = T.ar;   // the lane's row (same for its 4 slots)
    bool keep[4];
    uint32_t xs = 0, ys[4] = {0, 0, 0, 0};
    uint64_t mask[4];
    if constexpr (!EMIT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t cr = tb * kTile + (4 * lane + i) % kTile;
        keep[i] = ar < cr && cr < len;
        if (keep[i]) {
          xs = a.sids[p0 + ar];
          ys[i] = a.sids[p0 + cr];
          const uint32_t *kx = a.keys_om + size_t(xs) * a.n_bands;
          const uint32_t *ky = a.keys_om + size_t(ys[i]) * a.n_bands;
          for (int j = 0; j < a.band; ++j)   // collided in an earlier band: emitted there
            if (kx[j] == ky[j]) { keep[i] = false; break; }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) mask[i] = __ballot(keep[i]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mask[i] = a.tmask[4 * t + i];
        keep[i] = (mask[i] >> lane) & 1u;
        if (keep[i]) {
          const int64_t cr = tb * kTile + (4 * lane + i) % kTile;
          xs = a.sids[p0 + ar];
          ys[i] = a.sids[p0 + cr];
        }
      }
    }
    if (!EMIT) {
      int64_t total = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) total += __popcll(mask[i]);
      if (lane == 0) {
        a.tcnt[t] = total;
#pragma unroll
        for (int i = 0; i < 4; ++i) a.tmask[4 * t + i] = mask[i];
      }
    } else {
      int64_t rank = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) rank += lanes_below(mask[i]);
      const int64_t off = out0 + a.tcoff[t];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (keep[i]) {
          const int64_t pos = off + rank;
          if (pos < a.capacity) {
            a.x_out[pos] = xs;
            a.y_out[pos] = ys[i];
          }
          ++rank;
        }
      }
    }
  }
}

// The count pass for key rows whose length is a multiple of 4, up to band 16:
// each wave step takes two tiles, decodes both and issues both tiles' id and
// key loads before using any (a tile alone is a chain of dependent loads:
// tile offsets, member ids, key rows), comparing earlier-band keys 16 bytes
// at a time.  Same counts and ballots as k_band_tiles<false>.
__global__ __launch_bounds__(kBandBlock) void k_band_count_pairs(TileArgs a) {
  const int lane = lane_id();
  const int64_t waves = int64_t(gridDim.x) * (kBandBlock / kWave);
  const int64_t w0 = int64_t(blockIdx.x) * (kBandBlock / kWave) +
                     int64_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave));
  const int nq = (a.band + 3) >> 2;
  for (int64_t t0 = 2 * w0; t0 < a.n_tiles; t0 += 2 * waves) {
    TileAt T[2] = {tile_at(a, t0, lane), tile_at(a, t0 + 1, lane)};
    bool keep[2][4];
    uint32_t xs[2] = {0, 0}, ys[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (T[u].ok && T[u].ar < T[u].len) xs[u] = a.sids[T[u].p0 + T[u].ar];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t cr = T[u].tb * kTile + (4 * lane + i) % kTile;
        keep[u][i] = T[u].ok && T[u].ar < cr && cr < T[u].len;
        ys[u][i] = keep[u][i] ? a.sids[T[u].p0 + cr] : 0u;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (q < nq) {
        uint4 kx[2], ky[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          kx[u] = reinterpret_cast<const uint4 *>(a.keys_om + size_t(xs[u]) * a.n_bands)[q];
#pragma unroll
          for (int i = 0; i < 4; ++i)
            ky[u][i] = reinterpret_cast<const uint4 *>(a.keys_om + size_t(ys[u][i]) * a.n_bands)[q];
        }
        const int j = 4 * q;
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const uint4 x = kx[u], y = ky[u][i];
            if ((x.x == y.x && j < a.band) || (x.y == y.y && j + 1 < a.band) || (x.z == y.z && j + 2 < a.band) ||
                (x.w == y.w && j + 3 < a.band))
              keep[u][i] = false;
          }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      uint64_t mask[4];
      int64_t total = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mask[i] = __ballot(keep[u][i]);
        total += __popcll(mask[i]);
      }
      if (T[u].ok && lane == 0) {
        a.tcnt[t0 + u] = total;
#pragma unroll
        for (int i = 0; i < 4; ++i) a.tmask[4 * (t0 + u) + i] = mask[i];
      }
    }
  }
}

// Bit j of the low 16 bits of x moved to bit 4j.
__device__ inline uint64_t spread4(uint64_t x) {
  x &= 0xFFFFull;
  x = (x | (x << 24)) & 0x000000FF000000FFull;
  x = (x | (x << 12)) & 0x000F000F000F000Full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}

// Tile descriptors of a band (one thread per tile): the tile's first
// candidate index (the band's running pair count plus the tile's offset), its
// row and column counts and member ids (the band's sorted ids), and the keep
// mask in row-major bit order (the count pass's ballot i holds position
// 4l + i at bit l: word w of the mask takes lanes 16w .. 16w+15 of the four
// ballots, interleaved).
__global__ __launch_bounds__(kBandBlock) void k_band_tile_desc(TileArgs a, blsh_tile *out, int64_t out_base,
                                                               int64_t out_cap) {
  const int64_t t = int64_t(blockIdx.x) * kBandBlock + threadIdx.x;
  if (t >= a.n_tiles || out_base + t >= out_cap) return;
  const TileAt T = tile_at(a, t, 0);
  const int64_t ta = T.ar / kTile;
  blsh_tile d;
  d.first = *a.base + a.tcoff[t];
  d.n_rows = uint32_t(min<int64_t>(kTile, T.len - ta * kTile));
  d.n_cols = uint32_t(min<int64_t>(kTile, T.len - T.tb * kTile));
  const uint64_t b0 = a.tmask[4 * t], b1 = a.tmask[4 * t + 1], b2 = a.tmask[4 * t + 2], b3 = a.tmask[4 * t + 3];
#pragma unroll
  for (int w = 0; w < 4; ++w)
    d.keep[w] = spread4(b0 >> (16 * w)) | (spread4(b1 >> (16 * w)) << 1) | (spread4(b2 >> (16 * w)) << 2) |
                (spread4(b3 >> (16 * w)) << 3);
  for (int i = 0; i < kTile; ++i) {
    d.ids[i] = i < int(d.n_rows) ? a.sids[T.p0 + ta * kTile + i] : 0xFFFFFFFFu;
    d.ids[kTile + i] = i < int(d.n_cols) ? a.sids[T.p0 + T.tb * kTile + i] : 0xFFFFFFFFu;
  }
  for (int i = 0; i < 4; ++i) d.reserved[i] = 0;
  out[out_base + t] = d;
}

// base += (pairs of this band) = row_off[n-1] + row_count[n-1]
__global__ void k_band_advance(int64_t *base, const int64_t *row_off, const int64_t *row_count, int64_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && n > 0) *base += row_off[n - 1] + row_count[n - 1];
}

__global__ void k_band_zero(int64_t *base) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base = 0;
}

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static int ensure_tile_buf(blsh_ctx *ctx, size_t bytes) {
  if (ctx->tile_bytes >= bytes) return BLSH_OK;
  BLSH_HIP(hipDeviceSynchronize());
  if (ctx->tile_buf) (void)hipFree(ctx->tile_buf);
  ctx->tile_buf = nullptr;
  ctx->tile_bytes = 0;
  const size_t want = std::max(bytes, size_t(1) << 20);
  if (hipMalloc(&ctx->tile_buf, want) != hipSuccess) return fail(BLSH_ENOMEM, "banding: tile buffer of %zu bytes", want);
  ctx->tile_bytes = want;
  return BLSH_OK;
}

int band_candidates(blsh_ctx *ctx, const uint32_t *sig, int64_t n_obj, int32_t row_words, bool word_major,
                    int32_t n_bands, int32_t band_bits, int32_t max_bucket, int32_t tile, uint32_t *x_out,
                    uint32_t *y_out, int64_t capacity, int64_t *n_pairs, hipStream_t s, const BandTilesOut *to) {
  if (tile != 0 && tile != kTile) return fail(BLSH_EINVAL, "banding: order_tile must be 0 or %d", kTile);
  int64_t tiles_total = 0;   // tiles output: descriptors written so far (all bands)
  const size_t n = size_t(n_obj);
  // rocPRIM temporary storage sizes
  size_t sort_tmp = 0, scan_tmp = 0, flag_tmp = 0;
  if (rocprim::radix_sort_pairs(nullptr, sort_tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                (const uint32_t *)nullptr, (uint32_t *)nullptr, n, 0, unsigned(band_bits), s) !=
          hipSuccess ||
      rocprim::exclusive_scan(nullptr, scan_tmp, (const int64_t *)nullptr, (int64_t *)nullptr, int64_t(0), n,
                              rocprim::plus<int64_t>(), s) != hipSuccess ||
      rocprim::exclusive_scan(nullptr, flag_tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr, uint32_t(0), n,
                              rocprim::plus<uint32_t>(), s) != hipSuccess)
    return fail(BLSH_EDEVICE, "banding: temporary storage query failed");
  // workspace layout (row order: row counts and offsets; tiled order: the
  // same two int64 arrays hold tile counts and offsets per bucket)
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align256(bytes); return o; };
  const size_t o_kbm = take(n * n_bands * 4), o_kom = take(n * n_bands * 4), o_ids = take(n * 4),
               o_skeys = take(n * 4), o_sids = take(n * 4), o_bs = take(n * 4), o_be = take(n * 4),
               o_cnt = take(n * 8), o_off = take(n * 8), o_base = take(256),
               o_flag = take(tile ? n * 4 : 0), o_bidx = take(tile ? n * 4 : 0), o_bpos = take(tile ? n * 4 : 0),
               o_blen = take(tile ? n * 4 : 0), o_tmp = take(std::max({sort_tmp, scan_tmp, flag_tmp}));
  int rc = ensure_workspace(ctx, off);
  if (rc) return rc;
  char *ws = static_cast<char *>(ctx->ws);
  uint32_t *keys_bm = reinterpret_cast<uint32_t *>(ws + o_kbm), *keys_om = reinterpret_cast<uint32_t *>(ws + o_kom);
  uint32_t *ids = reinterpret_cast<uint32_t *>(ws + o_ids), *skeys = reinterpret_cast<uint32_t *>(ws + o_skeys);
  uint32_t *sids = reinterpret_cast<uint32_t *>(ws + o_sids);
  uint32_t *bstart = reinterpret_cast<uint32_t *>(ws + o_bs), *bend = reinterpret_cast<uint32_t *>(ws + o_be);
  int64_t *row_count = reinterpret_cast<int64_t *>(ws + o_cnt), *row_off = reinterpret_cast<int64_t *>(ws + o_off);
  int64_t *base = reinterpret_cast<int64_t *>(ws + o_base);
  int64_t *meta = base + 4;   // tiled order: bucket and tile totals of a band
  uint32_t *flag = reinterpret_cast<uint32_t *>(ws + o_flag), *bidx = reinterpret_cast<uint32_t *>(ws + o_bidx);
  uint32_t *bpos = reinterpret_cast<uint32_t *>(ws + o_bpos), *blen = reinterpret_cast<uint32_t *>(ws + o_blen);
  void *tmp = ws + o_tmp;

  LaunchScope ls(ctx, s, "band_candidates");
  const unsigned nb = unsigned((n + kBandBlock - 1) / kBandBlock);
  hipLaunchKernelGGL(k_band_keys, dim3(nb), dim3(kBandBlock), 0, s, sig, n_obj, row_words, int(word_major), n_bands,
                     band_bits, keys_bm, keys_om);
  hipLaunchKernelGGL(k_iota, dim3(nb), dim3(kBandBlock), 0, s, ids, n_obj);
  hipLaunchKernelGGL(k_band_zero, dim3(1), dim3(64), 0, s, base);
  const unsigned pair_blocks = unsigned(std::min<int64_t>(int64_t(ctx->n_cu) * 8, (n_obj + 3) / 4 + 1));
  for (int j = 0; j < n_bands; ++j) {
    size_t t1 = sort_tmp;
    if (rocprim::radix_sort_pairs(tmp, t1, keys_bm + size_t(j) * n, skeys, ids, sids, n, 0, unsigned(band_bits),
                                  s) != hipSuccess)
      return fail(BLSH_EDEVICE, "banding: radix sort failed");
    hipLaunchKernelGGL(k_bucket_bounds, dim3(nb), dim3(kBandBlock), 0, s, skeys, n_obj, bstart, bend);
    if (tile) {
      // buckets: index by a scan of start flags, then each bucket's tile count
      hipLaunchKernelGGL(k_start_flags, dim3(nb), dim3(kBandBlock), 0, s, bstart, n_obj, flag);
      size_t t2 = flag_tmp;
      if (rocprim::exclusive_scan(tmp, t2, flag, bidx, uint32_t(0), n, rocprim::plus<uint32_t>(), s) != hipSuccess)
        return fail(BLSH_EDEVICE, "banding: scan failed");
      hipLaunchKernelGGL(k_count_buckets, dim3(1), dim3(64), 0, s, flag, bidx, n_obj, meta);
      hipLaunchKernelGGL(k_bucket_tiles, dim3(nb), dim3(kBandBlock), 0, s, bstart, bend, bidx, n_obj, max_bucket,
                         bpos, blen, row_count);
      int64_t n_buckets = 0;
      BLSH_HIP(hipMemcpyAsync(&n_buckets, meta, 8, hipMemcpyDeviceToHost, s));
      BLSH_HIP(hipStreamSynchronize(s));
      size_t t3 = scan_tmp;
      if (rocprim::exclusive_scan(tmp, t3, row_count, row_off, int64_t(0), size_t(n_buckets),
                                  rocprim::plus<int64_t>(), s) != hipSuccess)
        return fail(BLSH_EDEVICE, "banding: scan failed");
      hipLaunchKernelGGL(k_count_tiles, dim3(1), dim3(64), 0, s, row_off, row_count, n_buckets, meta);
      int64_t n_tiles = 0;
      BLSH_HIP(hipMemcpyAsync(&n_tiles, meta + 1, 8, hipMemcpyDeviceToHost, s));
      BLSH_HIP(hipStreamSynchronize(s));
      if (n_tiles == 0) continue;
      // per-tile counts and offsets, and the scan's temporary storage
      size_t tile_tmp = 0;
      if (rocprim::exclusive_scan(nullptr, tile_tmp, (const int64_t *)nullptr, (int64_t *)nullptr, int64_t(0),
                                  size_t(n_tiles), rocprim::plus<int64_t>(), s) != hipSuccess)
        return fail(BLSH_EDEVICE, "banding: temporary storage query failed");
      const size_t tb = align256(size_t(n_tiles) * 8), mb = align256(size_t(n_tiles) * 32);
      if ((rc = ensure_tile_buf(ctx, 2 * tb + mb + tile_tmp))) return rc;
      int64_t *tcnt = static_cast<int64_t *>(ctx->tile_buf);
      int64_t *tcoff = reinterpret_cast<int64_t *>(static_cast<char *>(ctx->tile_buf) + tb);
      uint64_t *tmask = reinterpret_cast<uint64_t *>(static_cast<char *>(ctx->tile_buf) + 2 * tb);
      void *ttmp = static_cast<char *>(ctx->tile_buf) + 2 * tb + mb;
      TileArgs ta{};
      ta.sids = sids;
      ta.keys_om = keys_om;
      ta.n_bands = n_bands;
      ta.band = j;
      ta.bpos = bpos;
      ta.blen = blen;
      ta.toff = row_off;
      ta.n_buckets = n_buckets;
      ta.n_tiles = n_tiles;
      ta.tcnt = tcnt;
      ta.tmask = tmask;
      ta.tcoff = tcoff;
      ta.base = base;
      ta.x_out = x_out;
      ta.y_out = y_out;
      ta.capacity = capacity;
      const unsigned tile_blocks =
          unsigned(std::min<int64_t>(int64_t(ctx->n_cu) * 8, (n_tiles + kBandBlock / kWave - 1) / (kBandBlock / kWave)));
      if ((n_bands & 3) == 0 && j <= 16)
        hipLaunchKernelGGL(k_band_count_pairs, dim3(tile_blocks), dim3(kBandBlock), 0, s, ta);
      else
        hipLaunchKernelGGL(k_band_tiles<false>, dim3(tile_blocks), dim3(kBandBlock), 0, s, ta);
      size_t t4 = tile_tmp;
      if (rocprim::exclusive_scan(ttmp, t4, tcnt, tcoff, int64_t(0), size_t(n_tiles), rocprim::plus<int64_t>(), s) !=
          hipSuccess)
        return fail(BLSH_EDEVICE, "banding: scan failed");
      if (to) {   // tiles instead of pairs: this band's tile descriptors
        const unsigned db = unsigned((n_tiles + kBandBlock - 1) / kBandBlock);
        hipLaunchKernelGGL(k_band_tile_desc, dim3(db), dim3(kBandBlock), 0, s, ta, to->tiles, tiles_total,
                           to->tile_cap);
        tiles_total += n_tiles;
      } else {
        hipLaunchKernelGGL(k_band_tiles<true>, dim3(tile_blocks), dim3(kBandBlock), 0, s, ta);
      }
      hipLaunchKernelGGL(k_band_advance, dim3(1), dim3(64), 0, s, base, tcoff, tcnt, n_tiles);
      continue;
    }
    BandArgs a{};
    a.sids = sids;
    a.bstart = bstart;
    a.bend = bend;
    a.keys_om = keys_om;
    a.n_obj = n_obj;
    a.n_bands = n_bands;
    a.band = j;
    a.max_bucket = max_bucket;
    a.row_count = row_count;
    a.row_off = row_off;
    a.base = base;
    a.x_out = x_out;
    a.y_out = y_out;
    a.capacity = capacity;
    hipLaunchKernelGGL(k_band_pairs<false>, dim3(pair_blocks), dim3(kBandBlock), 0, s, a);
    size_t t2 = scan_tmp;
    if (rocprim::exclusive_scan(tmp, t2, row_count, row_off, int64_t(0), n, rocprim::plus<int64_t>(), s) !=
        hipSuccess)
      return fail(BLSH_EDEVICE, "banding: scan failed");
    hipLaunchKernelGGL(k_band_pairs<true>, dim3(pair_blocks), dim3(kBandBlock), 0, s, a);
    hipLaunchKernelGGL(k_band_advance, dim3(1), dim3(64), 0, s, base, row_off, row_count, n_obj);
  }
  BLSH_HIP(hipMemcpyAsync(n_pairs, base, 8, hipMemcpyDeviceToHost, s));
  BLSH_HIP(hipStreamSynchronize(s));
  if (hipGetLastError() != hipSuccess) return fail(BLSH_EDEVICE, "banding: launch failed");
  if (to) {
    *to->n_tiles = tiles_total;
    if (tiles_total > to->tile_cap)
      return fail(BLSH_ETRUNCATED, "banding: %lld tiles, capacity %lld", (long long)tiles_total,
                  (long long)to->tile_cap);
    return BLSH_OK;
  }
  return *n_pairs > capacity ? fail(BLSH_ETRUNCATED, "banding: %lld pairs, capacity %lld", (long long)*n_pairs,
                                    (long long)capacity)
                             : BLSH_OK;
}

}  // namespace blsh
