// Batched verification of many query lists of uneven lengths in one
// graph-launched pair of persistent kernels (Algorithm 1 per candidate).
//
// Phase 1 (k_batch_phase1, one launch per measure): the batch is cut into
//   wave tiles -- 128, 256 or 512 consecutive candidates of one SRP list (2, 4
//   or 8 per lane) or 64 or 128 of one minhash list (lane l owns candidates l
//   and 64 + l, a group of k/4 lanes compares each candidate's k hashes), the
//   shape per measure chosen by the autotuner -- and every wave of the fixed grid
//   runs one contiguous range of tiles (no work counter, no block barrier),
//   each XCD an eighth of every list (L2 locality of sorted ids).  The
//   query's hashes are wave-uniform.  Each list carries its own measure and
//   threshold, hence its own decision table, and each measure its own k.  A
//   candidate still undecided after `inreg_levels` levels (SRP object-major
//   rows: at least the 128 hashes one 16-byte load brings) is spilled to the
//   wave's own region of the measure's survivor queue (ballot compaction, no
//   atomics); when the region is full it simply continues in registers.
// Phase 2 (k_batch_phase2): persistent blocks drain the survivor queues with
//   every lane busy: one lane per SRP survivor (the words of the next levels
//   loaded ahead), one group of k/4 lanes per minhash survivor, running the
//   remaining levels; a block takes the regions it drains as one list.
//
// Accepted pairs are staged in slices (as in the single-call paths) and
// appended to the caller's list by k_batch_flush at the end of the batch.
//
// The kernels read all their arguments from one device-resident BatchBlock,
// so the graph that holds [reset, phase 1 x 2, phase 2, flush] is captured
// once per (k pair, tile shapes, grid) and replayed for any batch: each call
// only refreshes the block and the tile prefix sums.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <set>
#include <utility>

#include "device_common.h"

namespace blsh {

constexpr int kMaxBatchTables = 64;
constexpr int kBBlock = 256;
// phase 1 wave tiles (the autotuner picks one shape per measure):
// SRP 128, 256 or 512 consecutive candidates (2, 4 or 8 per lane), minhash 64
// or 128 (1 or 2 per lane)
constexpr int kSrpTileDefault = 256;
constexpr int kMhTileDefault = 64;
constexpr int kExSrpTile = 1024;   // comparator: candidates per SRP block tile
constexpr int kExMhTile = 256;     // comparator: candidates per minhash block tile
constexpr int kXcds = 8;           // phase 1: list tiles split in kXcds position ranges, one per XCD
constexpr int64_t kBatchStage = 4096;   // accepted-pair staging entries per slice

struct BatchList {
  int64_t offset;
  int64_t length;
  uint32_t query;
  int32_t measure;
  int32_t table;
  int32_t pad;
};

struct SigView {
  const uint32_t *data;
  int64_t n_obj;
  int32_t row_words;
  int32_t word_major;
  const uint32_t *pfx;          // SRP: hashes 0..127 of object i at pfx + i * pfx_stride, or null
  int64_t pfx_stride;
};

struct BatchBlock {
  const BatchList *lists;
  // phase 1: [2 measures][kXcds][n_lists + 1], slice (me, x) counts the
  // tiles [x n_t / kXcds, (x+1) n_t / kXcds) of each list of measure me (n_t
  // tiles); comparator: [n_lists + 1]
  const int64_t *tile_prefix;
  int64_t n_lists, n_tiles;
  const uint32_t *cand;
  SigView sig[2];               // [BLSH_JACCARD], [BLSH_COSINE]
  const uint32_t *tables[kMaxBatchTables];
  int32_t n_levels[kMaxBatchTables];
  double alpha, beta;           // Jaccard prior
  uint8_t *code;
  uint64_t *acc_idx;
  float *acc_val;
  int64_t acc_cap;
  int64_t *n_acc;
  uint16_t *m_dbg;
  int32_t *status;
  // accepted-pair staging (as in the single-call paths): kSlices slices of
  // st_cap entries, counts at acc_cnt[s * kCntStride], appended to the list by
  // k_batch_flush; entries past a slice's capacity go to the list directly at
  // positions from the running count *acc_total
  int64_t *acc_cnt;
  uint64_t *st_idx;
  float *st_val;
  int64_t st_cap;
  int64_t *acc_total;
  uint4 *spill[2];               // survivor queue per measure: spill_region entries per phase-1 wave
  uint32_t *spill_count[2];     // entries each phase-1 wave stored in its region
  int64_t spill_region;
  int32_t spill_waves;          // waves of the phase-1 grid
  int32_t inreg_levels;
};

// Spill entry: x = candidate position (low), y = candidate position (high),
// z = list index, w = m | level << 16 (level = next level to run).
__device__ inline uint4 spill_entry(int64_t pos, uint32_t list, uint32_t m, uint32_t next_level) {
  return make_uint4(uint32_t(pos), uint32_t(uint64_t(pos) >> 32), list, m | (next_level << 16));
}

// Read-only data (signatures, tables, list descriptors: nothing the kernels
// write) read through the constant address space, so that a wave-uniform
// address becomes one scalar load.
template <typename T>
__device__ inline T ld_uniform(const T *p) {
  return *(const __attribute__((address_space(4))) T *)(p);
}

__device__ inline BatchList ld_list(const BatchList *p) {
  BatchList r;
  r.offset = ld_uniform(&p->offset);
  r.length = ld_uniform(&p->length);
  r.query = ld_uniform(&p->query);
  r.measure = ld_uniform(&p->measure);
  r.table = ld_uniform(&p->table);
  r.pad = 0;
  return r;
}

template <int G, int... S>
__device__ inline void group_bcast_all(uint32_t v, uint32_t *out, std::integer_sequence<int, S...>) {
  ((out[S] = group_bcast<G, S>(v)), ...);
}

// Wave-level compaction of accepted pairs into the wave's staging slice (the
// list itself past the slice's capacity); called by all lanes of the wave.
__device__ inline void emit_block(const BatchBlock &B, bool pred, int64_t idx, float val) {
  uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  {
    const int sl = wave_slice();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader)
      base = atomicAdd((unsigned long long *)(B.acc_cnt + sl * kCntStride), (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    const unsigned long long pos = base + lanes_below(mask);
    if (pred && int64_t(pos) < B.st_cap) {
      B.st_idx[size_t(sl) * B.st_cap + pos] = uint64_t(idx);
      B.st_val[size_t(sl) * B.st_cap + pos] = val;
      pred = false;
    }
    mask = __ballot(pred);
    if (mask == 0) return;
  }
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd((unsigned long long *)B.acc_total, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) {
    const unsigned long long pos = base + lanes_below(mask);
    if (int64_t(pos) < B.acc_cap) {
      B.acc_idx[pos] = uint64_t(idx);
      B.acc_val[pos] = val;
    } else {
      raise_status(B.status, BLSH_ETRUNCATED);
    }
  }
}

// Survivor queue of a measure: phase-1 wave w owns the entries
// [w R, (w+1) R) (R = spill_region) and keeps its fill `n` in a register, so
// spilling takes a ballot and no atomic.  Bit p of `want`: the lane's
// candidate p; returns the bits whose entry was stored (the others found the
// region full and continue in registers).  Called by all lanes of the wave.
template <int P>
__device__ inline uint32_t spill_tile(const BatchBlock &B, int meas, int64_t wave, uint32_t &n, uint32_t want,
                                      const uint4 *e) {
  const int64_t R = B.spill_region;
  uint4 *region = B.spill[meas] + wave * R;
  uint32_t stored = 0;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const uint64_t mask = __ballot((want >> p) & 1u);
    if ((want >> p) & 1u) {
      const int64_t pos = int64_t(n) + lanes_below(mask);
      if (pos < R) {
        region[pos] = e[p];
        stored |= 1u << p;
      }
    }
    n = uint32_t(min<int64_t>(R, int64_t(n) + __popcll(mask)));
  }
  return stored;
}

template <int K>
__device__ inline uint32_t srp_level_word_agree(const SigView &s, uint32_t q, uint32_t y, int j) {
  auto word = [&](uint32_t id, int w) -> uint32_t {
    return s.word_major ? s.data[size_t(w) * s.n_obj + id] : s.data[size_t(id) * s.row_words + w];
  };
  if constexpr (K == 32) return 32u - __popc(word(q, j) ^ word(y, j));
  else if constexpr (K == 64) return 64u - __popc(word(q, 2 * j) ^ word(y, 2 * j)) - __popc(word(q, 2 * j + 1) ^ word(y, 2 * j + 1));
  else return 16u - __popc(((word(q, j >> 1) ^ word(y, j >> 1)) >> ((j & 1) * 16)) & 0xFFFFu);
}

// ---------------------------------------------------------------------------
// phase 1: wave tiles
// ---------------------------------------------------------------------------
// agreement of level j from the XOR of two 128-bit prefixes
template <int K>
__device__ inline uint32_t prefix_agree(const uint32_t *d, int j) {
  if constexpr (K == 32) return 32u - __popc(d[j]);
  else if constexpr (K == 64) return 64u - __popc(d[2 * j]) - __popc(d[2 * j + 1]);
  else return 16u - __popc((d[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu);
}

// 64 P consecutive candidates of one SRP list: candidate base + 64 p + lane.
template <int K, int P>
__device__ void srp_tile(const BatchBlock &B, const BatchList &Ls, int32_t list_id, int64_t base,
                         const uint32_t *tab, int L, int64_t wave, uint32_t &n_spill) {
  constexpr int PL = 128 / K;          // levels held by a 128-bit prefix
  const SigView S = B.sig[BLSH_COSINE];
  const int words = int(ld_uniform(tab + 2));
  const int lane = lane_id();
  const int64_t end = Ls.offset + Ls.length;
  const uint32_t q = Ls.query;
  const bool q_ok = q < S.n_obj;
  // a prefix view (the caller's prefix array, or object-major rows that a
  // 16-byte load can start): one gather per side serves the first 128 hashes
  const bool pfx = S.pfx != nullptr;
  uint32_t y[P], alive = 0, bad = 0, in = 0;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t c = base + p * kWave + lane;
    y[p] = 0;
    if (c < end) {
      in |= 1u << p;
      y[p] = __builtin_nontemporal_load(B.cand + c);
      if (q_ok && y[p] < S.n_obj) alive |= 1u << p; else { bad |= 1u << p; y[p] = 0; }
    }
  }
  uint32_t m[P], emit = 0;
  uint8_t code[P];
#pragma unroll
  for (int p = 0; p < P; ++p) { m[p] = 0; code[p] = 0; }
  auto decide = [&](int p, int j) {
    if (int(m[p]) < int(ld_uniform(tab + kTabMinOff + j))) {
      code[p] = uint8_t((BLSH_PRUNED << 6) | j);
      alive &= ~(1u << p);
    } else if (accept_bit(tab, words, j, int(m[p]))) {
      code[p] = uint8_t((BLSH_ACCEPT_CONC << 6) | j);
      alive &= ~(1u << p);
      emit |= 1u << p;
    } else if (j == L - 1) {
      code[p] = uint8_t((BLSH_ACCEPT_NMAX << 6) | j);
      alive &= ~(1u << p);
      emit |= 1u << p;
    }
  };
  auto word_levels = [&](int j0, int j1) {
    for (int j = j0; j < j1 && __ballot(alive != 0); ++j) {
#pragma unroll
      for (int p = 0; p < P; ++p)
        if (alive & (1u << p)) m[p] += srp_level_word_agree<K>(S, q, y[p], j);
#pragma unroll
      for (int p = 0; p < P; ++p)
        if (alive & (1u << p)) decide(p, j);
    }
  };
  const int J = min(L, max(B.inreg_levels, pfx ? PL : 0));
  int j = 0;
  if (pfx && __ballot(alive != 0)) {
    // all gathers issued before any is consumed; a lane without a live
    // candidate reads the query's own row
    const u32x4 hq = ld_uniform(reinterpret_cast<const u32x4 *>(S.pfx + size_t(q) * S.pfx_stride));
    u32x4 hy[P];
#pragma unroll
    for (int p = 0; p < P; ++p)
      hy[p] = *reinterpret_cast<const u32x4 *>(S.pfx + size_t((alive >> p) & 1u ? y[p] : q) * S.pfx_stride);
    uint32_t d[P][4];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      d[p][0] = hq.x ^ hy[p].x; d[p][1] = hq.y ^ hy[p].y;
      d[p][2] = hq.z ^ hy[p].z; d[p][3] = hq.w ^ hy[p].w;
    }
    const int JP = min(J, PL);
#pragma unroll
    for (int jj = 0; jj < PL; ++jj) {   // unrolled: d is indexed by constants
      if (jj < JP && __ballot(alive != 0)) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
          if (!(alive & (1u << p))) continue;
          m[p] += prefix_agree<K>(d[p], jj);
          decide(p, jj);
        }
      }
    }
    j = JP;
  }
  word_levels(j, J);
  // spill what is still undecided; what cannot be spilled continues here
  if (J < L) {
    uint4 e[P];
#pragma unroll
    for (int p = 0; p < P; ++p) e[p] = spill_entry(base + p * kWave + lane, uint32_t(list_id), m[p], uint32_t(J));
    alive &= ~spill_tile<P>(B, BLSH_COSINE, wave, n_spill, alive, e);
  }
  word_levels(J, L);
  if (bad) raise_status(B.status, BLSH_EBADID);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!((in >> p) & 1u)) continue;
    const int64_t c = base + p * kWave + lane;
    B.code[c] = (bad >> p) & 1u ? uint8_t(0xFF) : code[p];
    if (B.m_dbg) B.m_dbg[c] = uint16_t(m[p]);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const bool e = (emit >> p) & 1u;
    const float v = e ? map_estimate(BLSH_COSINE, int(m[p]), ((code[p] & 63) + 1) * K, 1.0, 1.0) : 0.f;
    emit_block(B, e, base + p * kWave + lane, v);
  }
}

// 64 P consecutive candidates of one minhash list: lane l owns candidates
// base + 64 p + l; the group of G = k/4 lanes holding a candidate compares the
// k hashes of each of its G members in turn (lane r holds hashes 4r..4r+3 of
// the level), with the rows of a pass loaded for all P candidates before any
// comparison.
template <int K, int P>
__device__ void minhash_tile(const BatchBlock &B, const BatchList &Ls, int32_t list_id, int64_t base,
                             const uint32_t *tab, int L, int64_t wave, uint32_t &n_spill) {
  constexpr int G = K / 4;
  constexpr int CH = G < 8 ? G : 8;      // rows in flight per pass and candidate
  const SigView S = B.sig[BLSH_JACCARD];
  const int words = int(ld_uniform(tab + 2));
  const int64_t end = Ls.offset + Ls.length;
  const int lane = lane_id(), r = lane & (G - 1);
  const uint32_t q = Ls.query;
  const bool q_ok = q < S.n_obj;
  uint32_t y[P], m[P], alive = 0, bad = 0, in = 0, emit = 0;
  uint8_t code[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t c = base + p * kWave + lane;
    y[p] = 0;
    m[p] = 0;
    code[p] = 0;
    if (c < end) {
      in |= 1u << p;
      y[p] = __builtin_nontemporal_load(B.cand + c);
      if (q_ok && y[p] < S.n_obj) alive |= 1u << p; else bad |= 1u << p;
    }
  }
  auto level = [&](int j) {
    // a lane whose candidate is decided (or invalid) reads the query's row
    uint32_t ys[P][G];
#pragma unroll
    for (int p = 0; p < P; ++p)
      group_bcast_all<G>((alive >> p) & 1u ? y[p] : q, ys[p], std::make_integer_sequence<int, G>{});
    const size_t col = size_t(j) * K + 4 * r;
    const uint4 hq = *reinterpret_cast<const uint4 *>(S.data + size_t(q) * S.row_words + col);
    uint32_t own[P];
#pragma unroll
    for (int p = 0; p < P; ++p) own[p] = 0;
#pragma unroll
    for (int s0 = 0; s0 < G; s0 += CH) {
      uint4 hy[P][CH];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int s = 0; s < CH; ++s)
          hy[p][s] = *reinterpret_cast<const uint4 *>(S.data + size_t(ys[p][s0 + s]) * S.row_words + col);
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int s = 0; s < CH; ++s) {
          uint32_t cnt = uint32_t(hq.x == hy[p][s].x) + uint32_t(hq.y == hy[p][s].y) +
                         uint32_t(hq.z == hy[p][s].z) + uint32_t(hq.w == hy[p][s].w);
          cnt = group_sum<G>(cnt);
          if (r == s0 + s) own[p] = cnt;
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (!((alive >> p) & 1u)) continue;
      m[p] += own[p];
      const int mp = int(m[p]);
      if (mp < int(ld_uniform(tab + kTabMinOff + j))) {
        code[p] = uint8_t((BLSH_PRUNED << 6) | j);
        alive &= ~(1u << p);
      } else if (accept_bit(tab, words, j, mp)) {
        code[p] = uint8_t((BLSH_ACCEPT_CONC << 6) | j);
        alive &= ~(1u << p);
        emit |= 1u << p;
      } else if (j == L - 1) {
        code[p] = uint8_t((BLSH_ACCEPT_NMAX << 6) | j);
        alive &= ~(1u << p);
        emit |= 1u << p;
      }
    }
  };
  const int J = min(L, B.inreg_levels);
  for (int j = 0; j < J && __ballot(alive != 0); ++j) level(j);
  if (J < L) {
    uint4 e[P];
#pragma unroll
    for (int p = 0; p < P; ++p) e[p] = spill_entry(base + p * kWave + lane, uint32_t(list_id), m[p], uint32_t(J));
    alive &= ~spill_tile<P>(B, BLSH_JACCARD, wave, n_spill, alive, e);
  }
  for (int j = J; j < L && __ballot(alive != 0); ++j) level(j);
  if (bad) raise_status(B.status, BLSH_EBADID);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!((in >> p) & 1u)) continue;
    const int64_t c = base + p * kWave + lane;
    B.code[c] = (bad >> p) & 1u ? uint8_t(0xFF) : code[p];
    if (B.m_dbg) B.m_dbg[c] = uint16_t(m[p]);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const bool e = (emit >> p) & 1u;
    const float v = e ? map_estimate(BLSH_JACCARD, int(m[p]), ((code[p] & 63) + 1) * K, B.alpha, B.beta) : 0.f;
    emit_block(B, e, base + p * kWave + lane, v);
  }
}

// Index of the list holding tile t (the last l with prefix[l] <= t).
__device__ inline int64_t list_of_tile(const int64_t *prefix, int64_t n_lists, int64_t t) {
  int64_t lo = 0, hi = n_lists - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ld_uniform(prefix + mid) <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The tiles [t0, t1) of slice x, run in order by one wave (lists of measure
// MEAS, 64 P candidates per tile).
template <int MEAS, int K, int P>
__device__ inline void phase1_range(const BatchBlock &B, int x, const int64_t *prefix, int64_t t0, int64_t t1,
                                    int64_t wave, uint32_t &n_spill) {
  constexpr int64_t tsz = int64_t(P) * kWave;
  int64_t l = list_of_tile(prefix, B.n_lists, t0);
  int64_t first = ld_uniform(prefix + l), next = ld_uniform(prefix + l + 1);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= next) {   // lists with no tiles in this slice
      ++l;
      first = next;
      next = ld_uniform(prefix + l + 1);
    }
    const BatchList Ls = ld_list(B.lists + l);
    const uint32_t *tab = ld_uniform(B.tables + Ls.table);
    const int L = ld_uniform(B.n_levels + Ls.table);
    const int64_t tile = (int64_t(x) * ((Ls.length + tsz - 1) / tsz)) / kXcds + (t - first);
    if constexpr (MEAS == BLSH_COSINE)
      srp_tile<K, P>(B, Ls, int32_t(l), Ls.offset + tile * tsz, tab, L, wave, n_spill);
    else
      minhash_tile<K, P>(B, Ls, int32_t(l), Ls.offset + tile * tsz, tab, L, wave, n_spill);
  }
}

// Blocks are dealt round-robin over the XCDs (block b runs on XCD b mod 8),
// each with its own L2.  Phase 1 gives the blocks of XCD x the x-th eighth
// (by position) of every list's tiles: lists hold sorted candidate ids, so an
// XCD touches about an eighth of the signature rows and its L2 holds them.
// Within an XCD every wave runs a contiguous range of that XCD's tiles.  One
// launch runs the lists of one measure (MEAS), so the streaming minhash rows
// do not evict the SRP rows from L2.
template <int MEAS, int K, int P>
__global__ __launch_bounds__(kBBlock) void k_batch_phase1(const BatchBlock *__restrict__ Bp) {
  const BatchBlock &B = *Bp;
  const int x = int(blockIdx.x) % kXcds;
  const int64_t nbx = (int64_t(gridDim.x) - x + kXcds - 1) / kXcds;      // blocks on this XCD (grid >= kXcds)
  const int64_t wx = int64_t(blockIdx.x / kXcds) * (kBBlock / kWave) +
                     int64_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave));
  const int64_t Wx = nbx * (kBBlock / kWave);
  const int64_t *prefix = B.tile_prefix + int64_t(MEAS * kXcds + x) * (B.n_lists + 1);
  const int64_t Tx = ld_uniform(prefix + B.n_lists);
  const int64_t t0 = wx * Tx / Wx, t1 = (wx + 1) * Tx / Wx;
  const int64_t wave = int64_t(blockIdx.x) * (kBBlock / kWave) +
                       int64_t(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave));
  uint32_t n_spill = 0;
  if (t0 < t1) phase1_range<MEAS, K, P>(B, x, prefix, t0, t1, wave, n_spill);
  if (lane_id() == 0)   // every wave of the grid reports its fill, 0 included
    B.spill_count[MEAS][wave] = n_spill;
}

// ---------------------------------------------------------------------------
// phase 2: spilled survivors
// ---------------------------------------------------------------------------
// Block b drains the regions of phase-1 waves b, b + grid, ... taken together
// as one list: a region holds few survivors, and each survivor is a chain of
// dependent level loads, so passes over the concatenation overlap the chains
// of all its regions.  Item i of that list: its wave and its entry there.
__device__ inline bool region_item(const uint32_t *count, int64_t n_waves, int64_t i, int64_t &w_out,
                                   int64_t &k_out) {
  int64_t acc = 0;
  for (int64_t w = blockIdx.x; w < n_waves; w += gridDim.x) {
    const int64_t n = count[w];
    if (i < acc + n) {
      w_out = w;
      k_out = i - acc;
      return true;
    }
    acc += n;
  }
  return false;
}

__device__ inline int64_t block_region_total(const uint32_t *count, int64_t n_waves) {
  int64_t t = 0;
  for (int64_t w = blockIdx.x; w < n_waves; w += gridDim.x) t += count[w];
  return t;
}

// SRP words of level j of q and y (k = 16: the word holding the level)
template <int K>
struct LevelWords {
  uint32_t q[K == 64 ? 2 : 1], y[K == 64 ? 2 : 1];
};
template <int K>
__device__ inline void load_level(const SigView &s, uint32_t q, uint32_t y, int j, LevelWords<K> &w) {
  auto word = [&](uint32_t id, int i) -> uint32_t {
    return s.word_major ? s.data[size_t(i) * s.n_obj + id] : s.data[size_t(id) * s.row_words + i];
  };
  if constexpr (K == 64) {
    w.q[0] = word(q, 2 * j);
    w.q[1] = word(q, 2 * j + 1);
    w.y[0] = word(y, 2 * j);
    w.y[1] = word(y, 2 * j + 1);
  } else {
    const int i = K == 32 ? j : j >> 1;
    w.q[0] = word(q, i);
    w.y[0] = word(y, i);
  }
}
template <int K>
__device__ inline uint32_t level_agree(const LevelWords<K> &w, int j) {
  if constexpr (K == 64) return 64u - __popc(w.q[0] ^ w.y[0]) - __popc(w.q[1] ^ w.y[1]);
  else if constexpr (K == 32) return 32u - __popc(w.q[0] ^ w.y[0]);
  else return 16u - __popc(((w.q[0] ^ w.y[0]) >> ((j & 1) * 16)) & 0xFFFFu);
}

// SRP levels whose words are loaded before the first of them is decided: four
// shorten the chain of a deep survivor (dense serving 50 -> 41 ms); at k = 64
// a level is already two words per side and the loads past the decision cost
// more than they save.
template <int K>
constexpr int phase2_ahead() { return K == 64 ? 1 : 4; }

template <int KJ, int KC>
__global__ __launch_bounds__(kBBlock) void k_batch_phase2(const BatchBlock *__restrict__ Bp) {
  constexpr int G = KJ / 4;
  constexpr int AHEAD = phase2_ahead<KC>();
  const BatchBlock &B = *Bp;
  const int64_t R = B.spill_region;
  // SRP survivors: one lane each
  {
    const SigView &S = B.sig[BLSH_COSINE];
    const uint32_t *cnt = B.spill_count[BLSH_COSINE];
    const int64_t total = block_region_total(cnt, B.spill_waves);
    for (int64_t i0 = 0; i0 < total; i0 += kBBlock) {
      int64_t w = 0, k = 0;
      const bool act = region_item(cnt, B.spill_waves, i0 + threadIdx.x, w, k);
      int64_t pos = 0;
      uint32_t m = 0;
      uint8_t code = 0;
      bool emit = false;
      if (act) {
        const uint4 e = B.spill[BLSH_COSINE][w * R + k];
        pos = int64_t(uint64_t(e.x) | (uint64_t(e.y) << 32));
        const BatchList Ls = B.lists[e.z];
        const uint32_t *tab = B.tables[Ls.table];
        const int L = B.n_levels[Ls.table];
        const int words = int(tab[2]);
        m = e.w & 0xFFFFu;
        const uint32_t q = Ls.query, yv = B.cand[pos];
        bool done = false;
        for (int j0 = int(e.w >> 16); j0 < L && !done; j0 += AHEAD) {
          LevelWords<KC> lw[AHEAD];
#pragma unroll
          for (int d = 0; d < AHEAD; ++d)
            if (j0 + d < L) load_level<KC>(S, q, yv, j0 + d, lw[d]);
#pragma unroll
          for (int d = 0; d < AHEAD; ++d) {
            const int j = j0 + d;
            if (done || j >= L) break;
            m += level_agree<KC>(lw[d], j);
            if (int(m) < int(tab[kTabMinOff + j])) { code = uint8_t((BLSH_PRUNED << 6) | j); done = true; }
            else if (accept_bit(tab, words, j, int(m))) { code = uint8_t((BLSH_ACCEPT_CONC << 6) | j); emit = true; done = true; }
            else if (j == L - 1) { code = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); emit = true; done = true; }
          }
        }
        B.code[pos] = code;
        if (B.m_dbg) B.m_dbg[pos] = uint16_t(m);
      }
      const float v = emit ? map_estimate(BLSH_COSINE, int(m), ((code & 63) + 1) * KC, 1.0, 1.0) : 0.f;
      emit_block(B, emit, pos, v);
    }
  }
  // minhash survivors: one group of G lanes each
  {
    const SigView &S = B.sig[BLSH_JACCARD];
    const uint32_t *cnt = B.spill_count[BLSH_JACCARD];
    const int64_t total = block_region_total(cnt, B.spill_waves);
    constexpr int PER_BLOCK = kBBlock / G;
    const int g = threadIdx.x / G, r = threadIdx.x % G;
    for (int64_t i0 = 0; i0 < total; i0 += PER_BLOCK) {
      int64_t w = 0, k = 0;
      const bool act = region_item(cnt, B.spill_waves, i0 + g, w, k);
      int64_t pos = 0;
      uint32_t m = 0, q = 0, yv = 0;
      int j = 0, L = 0, words = 0;
      const uint32_t *tab = nullptr;
      if (act) {
        const uint4 e = B.spill[BLSH_JACCARD][w * R + k];
        pos = int64_t(uint64_t(e.x) | (uint64_t(e.y) << 32));
        const BatchList Ls = B.lists[e.z];
        tab = B.tables[Ls.table];
        L = B.n_levels[Ls.table];
        words = int(tab[2]);
        m = e.w & 0xFFFFu;
        j = int(e.w >> 16);
        q = Ls.query;
        yv = B.cand[pos];
      }
      bool alive = act && j < L;
      uint8_t code = 0;
      bool emit = false;
      while (__ballot(alive) != 0) {
        uint32_t c = 0;
        if (alive) {
          const uint4 hq = *reinterpret_cast<const uint4 *>(S.data + size_t(q) * S.row_words + j * KJ + 4 * r);
          const uint4 hy = *reinterpret_cast<const uint4 *>(S.data + size_t(yv) * S.row_words + j * KJ + 4 * r);
          c = uint32_t(hq.x == hy.x) + uint32_t(hq.y == hy.y) + uint32_t(hq.z == hy.z) + uint32_t(hq.w == hy.w);
        }
        c = group_sum<G>(c);
        if (alive) {
          m += c;
          if (int(m) < int(tab[kTabMinOff + j])) { code = uint8_t((BLSH_PRUNED << 6) | j); alive = false; }
          else if (accept_bit(tab, words, j, int(m))) { code = uint8_t((BLSH_ACCEPT_CONC << 6) | j); emit = true; alive = false; }
          else if (j == L - 1) { code = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); emit = true; alive = false; }
          ++j;
        }
      }
      if (act && r == 0) {
        B.code[pos] = code;
        if (B.m_dbg) B.m_dbg[pos] = uint16_t(m);
      }
      const bool e = emit && r == 0;
      const float v = e ? map_estimate(BLSH_JACCARD, int(m), ((code & 63) + 1) * KJ, B.alpha, B.beta) : 0.f;
      emit_block(B, e, pos, v);
    }
  }
}

// ---------------------------------------------------------------------------
// exhaustive comparator over the same tiles: every candidate compares the
// full n_max hashes of its row with the query's, and the decision sequence of
// Algorithm 1 is replayed on the per-level counts (same output).
// ---------------------------------------------------------------------------
// first level in [j0, j1) at which the running count decides; updates m
__device__ inline int replay_level(const uint32_t *tab, int words, int L, int j, int m, uint8_t &code) {
  if (m < int(tab[kTabMinOff + j])) { code = uint8_t((BLSH_PRUNED << 6) | j); return 1; }
  if (accept_bit(tab, words, j, m)) { code = uint8_t((BLSH_ACCEPT_CONC << 6) | j); return 2; }
  if (j == L - 1) { code = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); return 2; }
  return 0;
}

// SRP rows of W words: groups of G = W/4 lanes per candidate (one 16-byte load
// per lane), exclusive prefix of lane totals, first deciding lane by ballot.
template <int K, int G>
__device__ void srp_tile_exhaustive(const BatchBlock &B, const BatchList &Ls, int64_t tile_in_list,
                                    const uint32_t *tab, int L) {
  constexpr int LPL = 128 / K;                 // levels per lane
  constexpr int PER_BLOCK = kBBlock / G;
  const SigView &S = B.sig[BLSH_COSINE];
  const int words = int(tab[2]);
  const int lane = lane_id(), r = lane % G, g = threadIdx.x / G, gw = lane / G;
  const int64_t end = Ls.offset + Ls.length;
  const uint32_t q = Ls.query;
  const bool q_ok = q < S.n_obj;
  uint4 hq = make_uint4(0, 0, 0, 0);
  if (q_ok) hq = *reinterpret_cast<const uint4 *>(S.data + size_t(q) * S.row_words + 4 * r);
  const int64_t t0 = Ls.offset + tile_in_list * kExSrpTile;
  for (int64_t c0 = t0; c0 < min(end, t0 + kExSrpTile); c0 += PER_BLOCK) {
    const int64_t c = c0 + g;
    const bool in = c < end;
    uint32_t y = 0;
    bool ok = false;
    if (in) {
      y = B.cand[c];
      ok = q_ok && y < S.n_obj;
    }
    uint32_t cnt[LPL], tot = 0;
    if (ok) {
      const uint4 hy = *reinterpret_cast<const uint4 *>(S.data + size_t(y) * S.row_words + 4 * r);
      const uint32_t d[4] = {hq.x ^ hy.x, hq.y ^ hy.y, hq.z ^ hy.z, hq.w ^ hy.w};
#pragma unroll
      for (int qq = 0; qq < LPL; ++qq) {
        if constexpr (K == 16) cnt[qq] = 16u - __popc((d[qq >> 1] >> ((qq & 1) * 16)) & 0xFFFFu);
        else if constexpr (K == 32) cnt[qq] = 32u - __popc(d[qq]);
        else cnt[qq] = 64u - __popc(d[2 * qq]) - __popc(d[2 * qq + 1]);
        tot += cnt[qq];
      }
    } else {
#pragma unroll
      for (int qq = 0; qq < LPL; ++qq) cnt[qq] = 0;
    }
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const uint32_t v = __shfl_up(incl, o, G);
      if (r >= o) incl += v;
    }
    uint32_t run = incl - tot;
    int dec = 0, dm = 0;
    uint8_t dcode = 0;
#pragma unroll
    for (int qq = 0; qq < LPL; ++qq) {
      run += cnt[qq];
      const int j = r * LPL + qq;
      uint8_t cd;
      if (!dec && ok && j < L) {
        const int rr = replay_level(tab, words, L, j, int(run), cd);
        if (rr) { dec = rr; dm = int(run); dcode = cd; }
      }
    }
    const uint64_t has = __ballot(dec != 0);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (gw * G);
    const uint64_t mine = has & gmask;
    const int first = mine ? __ffsll((unsigned long long)mine) - 1 : gw * G;
    const int fdec = __shfl(dec, first), fm = __shfl(dm, first);
    const uint32_t fcode = __shfl(uint32_t(dcode), first);
    bool emit = false;
    if (in && r == 0) {
      B.code[c] = ok ? uint8_t(fcode) : uint8_t(0xFF);
      if (B.m_dbg) B.m_dbg[c] = uint16_t(fm);
      emit = ok && fdec == 2;
      if (!ok) raise_status(B.status, BLSH_EBADID);
    }
    const float v = emit ? map_estimate(BLSH_COSINE, fm, ((fcode & 63) + 1) * K, 1.0, 1.0) : 0.f;
    emit_block(B, emit, c, v);
  }
}

// Minhash rows: groups of 16 lanes per candidate, 64 hashes (256 B) per pass;
// per-level sums with DPP, then the levels replayed in order.
template <int K>
__device__ void minhash_tile_exhaustive(const BatchBlock &B, const BatchList &Ls, int64_t tile_in_list,
                                        const uint32_t *tab, int L, int H) {
  constexpr int G = 16;
  constexpr int LPC = 64 / K;                  // levels per 64-hash chunk
  constexpr int LL = K / 4;                    // lanes per level
  constexpr int PER_BLOCK = kBBlock / G;
  const SigView &S = B.sig[BLSH_JACCARD];
  const int words = int(tab[2]);
  const int lane = lane_id(), r = lane % G, g = threadIdx.x / G, gw = lane / G;
  const int64_t end = Ls.offset + Ls.length;
  const uint32_t q = Ls.query;
  const bool q_ok = q < S.n_obj;
  const int64_t t0 = Ls.offset + tile_in_list * kExMhTile;
  for (int64_t c0 = t0; c0 < min(end, t0 + kExMhTile); c0 += PER_BLOCK) {
    const int64_t c = c0 + g;
    const bool in = c < end;
    uint32_t y = 0;
    bool ok = false;
    if (in) {
      y = B.cand[c];
      ok = q_ok && y < S.n_obj;
    }
    int m = 0, dec = 0, dm = 0;
    uint8_t dcode = 0;
    for (int h0 = 0; h0 < H; h0 += 64) {
      uint32_t cnt = 0;
      if (ok) {
        const uint4 hq = *reinterpret_cast<const uint4 *>(S.data + size_t(q) * S.row_words + h0 + 4 * r);
        const uint4 hy = *reinterpret_cast<const uint4 *>(S.data + size_t(y) * S.row_words + h0 + 4 * r);
        cnt = uint32_t(hq.x == hy.x) + uint32_t(hq.y == hy.y) + uint32_t(hq.z == hy.z) + uint32_t(hq.w == hy.w);
      }
      cnt = group_sum<LL>(cnt);
#pragma unroll
      for (int sl = 0; sl < LPC; ++sl) {
        const uint32_t lev = __shfl(cnt, gw * G + sl * LL);
        m += int(lev);
        const int j = h0 / K + sl;
        uint8_t cd;
        if (!dec && ok && j < L) {
          const int rr = replay_level(tab, words, L, j, m, cd);
          if (rr) { dec = rr; dm = m; dcode = cd; }
        }
      }
    }
    bool emit = false;
    if (in && r == 0) {
      B.code[c] = ok ? dcode : uint8_t(0xFF);
      if (B.m_dbg) B.m_dbg[c] = uint16_t(dm);
      emit = ok && dec == 2;
      if (!ok) raise_status(B.status, BLSH_EBADID);
    }
    const float v = emit ? map_estimate(BLSH_JACCARD, dm, ((dcode & 63) + 1) * K, B.alpha, B.beta) : 0.f;
    emit_block(B, emit, c, v);
  }
}

// Block b of the fixed grid runs the block tiles [b T / NB, (b+1) T / NB).
template <int KJ, int KC>
__global__ __launch_bounds__(kBBlock) void k_batch_exhaustive(const BatchBlock *__restrict__ Bp) {
  const BatchBlock &B = *Bp;
  const int64_t T = B.n_tiles, NB = gridDim.x;
  const int64_t t0 = int64_t(blockIdx.x) * T / NB, t1 = (int64_t(blockIdx.x) + 1) * T / NB;
  if (t0 >= t1) return;
  int64_t l = list_of_tile(B.tile_prefix, B.n_lists, t0);
  int64_t first = ld_uniform(B.tile_prefix + l), next = ld_uniform(B.tile_prefix + l + 1);
  for (int64_t t = t0; t < t1; ++t) {
    while (t >= next) {
      ++l;
      first = next;
      next = ld_uniform(B.tile_prefix + l + 1);
    }
    const BatchList Ls = ld_list(B.lists + l);
    const uint32_t *tab = ld_uniform(B.tables + Ls.table);
    const int L = ld_uniform(B.n_levels + Ls.table);
    const int64_t tl = t - first;
    if (Ls.measure == BLSH_COSINE) {
      const int W = L * KC / 32;   // words compared: n_max bits
      if (W == 4) srp_tile_exhaustive<KC, 1>(B, Ls, tl, tab, L);
      else if (W == 8) srp_tile_exhaustive<KC, 2>(B, Ls, tl, tab, L);
      else if (W == 16) srp_tile_exhaustive<KC, 4>(B, Ls, tl, tab, L);
      else if (W == 32) srp_tile_exhaustive<KC, 8>(B, Ls, tl, tab, L);
      else srp_tile_exhaustive<KC, 16>(B, Ls, tl, tab, L);
    } else {
      minhash_tile_exhaustive<KJ>(B, Ls, tl, tab, L, L * KJ);
    }
  }
}

// Clears the running count and the staging counts: one block of kSlices
// threads.
__global__ void k_batch_reset(const BatchBlock *__restrict__ Bp) {
  const BatchBlock &B = *Bp;
  B.acc_cnt[threadIdx.x * kCntStride] = 0;
  if (threadIdx.x == 0) *B.acc_total = 0;
}

// Appends the staging slices to the accepted list, one block per slice, no
// atomics: every block scans the kSlices counts, block s copies slice s after
// the slices before it and after the entries written directly; block 0
// stores the final count to *n_acc (which no block reads).
__global__ __launch_bounds__(kBBlock) void k_batch_flush(const BatchBlock *__restrict__ Bp) {
  static_assert(kSlices == kBBlock, "one staging slice per thread of a block");
  const BatchBlock &B = *Bp;
  __shared__ int64_t s_cnt[kSlices];
  __shared__ int64_t s_base, s_total;
  const int t = threadIdx.x, sl = blockIdx.x;
  const int64_t c = min(B.acc_cnt[size_t(t) * kCntStride], B.st_cap);
  int64_t v = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t u = __shfl_up(v, o);
    if (lane_id() >= o) v += u;
  }
  s_cnt[t] = v;
  __syncthreads();
  int64_t before = 0;
  for (int w = 0; w < (t >> 6); ++w) before += s_cnt[w * kWave + kWave - 1];
  __syncthreads();
  s_cnt[t] = before + v - c;
  if (t == kSlices - 1) s_total = before + v;
  if (t == 0) s_base = *B.acc_total;
  __syncthreads();
  const int64_t n = min(B.acc_cnt[size_t(sl) * kCntStride], B.st_cap);
  const int64_t base = s_base + s_cnt[sl];
  const uint64_t *idx = B.st_idx + size_t(sl) * B.st_cap;
  const float *val = B.st_val + size_t(sl) * B.st_cap;
  bool trunc = false;
  for (int64_t i = t; i < n; i += kBBlock) {
    const int64_t pos = base + i;
    if (pos < B.acc_cap) {
      B.acc_idx[pos] = idx[i];
      B.acc_val[pos] = val[i];
    } else {
      trunc = true;
    }
  }
  if (trunc) raise_status(B.status, BLSH_ETRUNCATED);
  if (sl == 0 && t == 0) *B.n_acc = s_base + s_total;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchState {
  BatchBlock *d_block = nullptr;
  BatchBlock *h_block = nullptr;        // pinned staging
  BatchList *d_lists = nullptr, *h_lists = nullptr;
  int64_t *d_prefix = nullptr, *h_prefix = nullptr;
  int64_t lists_cap = 0;
  // staging: kSlices counters (kCntStride apart), the running count, then
  // kSlices x kBatchStage entries
  int64_t *d_stage_cnt = nullptr;
  uint64_t *d_st_idx = nullptr;
  float *d_st_val = nullptr;
  uint4 *d_spill[2] = {nullptr, nullptr};
  int64_t spill_cap = 0;
  uint32_t *d_spill_count = nullptr;    // [2][spill_waves_cap]
  int64_t spill_waves_cap = 0;
  hipEvent_t staged{};
  bool staged_valid = false;
  hipStream_t cap_stream{};
  struct GraphKey {
    int mode, kj, kc, ts, tm, grid1, grid2;
    bool operator<(const GraphKey &o) const {
      return std::tie(mode, kj, kc, ts, tm, grid1, grid2) < std::tie(o.mode, o.kj, o.kc, o.ts, o.tm, o.grid1, o.grid2);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  // k per measure, SRP / minhash tile (candidates per wave tile), in-register
  // levels, blocks per CU
  struct Choice { int kj, kc, ts, tm, inreg, bpc; };
  std::map<std::vector<int64_t>, Choice> tuned;
};

static void batch_free(BatchState *b) {
  if (!b) return;
  for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
  if (b->d_block) (void)hipFree(b->d_block);
  if (b->h_block) (void)hipHostFree(b->h_block);
  if (b->d_lists) (void)hipFree(b->d_lists);
  if (b->h_lists) (void)hipHostFree(b->h_lists);
  if (b->d_prefix) (void)hipFree(b->d_prefix);
  if (b->h_prefix) (void)hipHostFree(b->h_prefix);
  if (b->d_stage_cnt) (void)hipFree(b->d_stage_cnt);
  if (b->d_st_idx) (void)hipFree(b->d_st_idx);
  if (b->d_st_val) (void)hipFree(b->d_st_val);
  for (auto *p : b->d_spill) if (p) (void)hipFree(p);
  if (b->d_spill_count) (void)hipFree(b->d_spill_count);
  if (b->staged_valid) (void)hipEventDestroy(b->staged);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

void batch_state_free(void *p) { batch_free(static_cast<BatchState *>(p)); }

static int batch_state(blsh_ctx *ctx, BatchState **out) {
  if (!ctx->batch) {
    auto *b = new (std::nothrow) BatchState();
    if (!b) return fail(BLSH_ENOMEM, "host allocation failed");
    if (hipMalloc(&b->d_block, sizeof(BatchBlock)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&b->h_block), sizeof(BatchBlock), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&b->d_stage_cnt, (size_t(kSlices) + 1) * kCntStride * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&b->d_st_idx, size_t(kSlices) * kBatchStage * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&b->d_st_val, size_t(kSlices) * kBatchStage * sizeof(float)) != hipSuccess ||
        hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return fail(BLSH_ENOMEM, "batched state allocation failed");
    }
    b->staged_valid = true;
    ctx->batch = b;
    ctx->batch_free = batch_state_free;
  }
  *out = static_cast<BatchState *>(ctx->batch);
  return BLSH_OK;
}

static int grow_lists(BatchState *b, int64_t n_lists) {
  if (b->lists_cap >= n_lists) return BLSH_OK;
  BLSH_HIP(hipDeviceSynchronize());
  if (b->d_lists) (void)hipFree(b->d_lists);
  if (b->h_lists) (void)hipHostFree(b->h_lists);
  if (b->d_prefix) (void)hipFree(b->d_prefix);
  if (b->h_prefix) (void)hipHostFree(b->h_prefix);
  b->d_lists = b->h_lists = nullptr;
  b->d_prefix = b->h_prefix = nullptr;
  b->lists_cap = 0;
  const int64_t cap = std::max<int64_t>(n_lists, 1024);
  if (hipMalloc(&b->d_lists, cap * sizeof(BatchList)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&b->h_lists), cap * sizeof(BatchList), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&b->d_prefix, 2 * kXcds * (cap + 1) * sizeof(int64_t)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&b->h_prefix), 2 * kXcds * (cap + 1) * sizeof(int64_t),
                    hipHostMallocDefault) != hipSuccess)
    return fail(BLSH_ENOMEM, "list buffers");
  b->lists_cap = cap;
  return BLSH_OK;
}

static int grow_spill_counts(BatchState *b, int64_t waves) {
  if (b->spill_waves_cap >= waves) return BLSH_OK;
  BLSH_HIP(hipDeviceSynchronize());
  if (b->d_spill_count) (void)hipFree(b->d_spill_count);
  b->d_spill_count = nullptr;
  b->spill_waves_cap = 0;
  if (hipMalloc(&b->d_spill_count, size_t(2 * waves) * sizeof(uint32_t)) != hipSuccess)
    return fail(BLSH_ENOMEM, "spill counts");
  b->spill_waves_cap = waves;
  return BLSH_OK;
}

static int grow_spill(BatchState *b, int64_t cap) {
  if (b->spill_cap >= cap) return BLSH_OK;
  BLSH_HIP(hipDeviceSynchronize());
  for (auto *&p : b->d_spill) { if (p) (void)hipFree(p); p = nullptr; }
  b->spill_cap = 0;
  for (auto *&p : b->d_spill)
    if (hipMalloc(&p, size_t(cap) * sizeof(uint4)) != hipSuccess) return fail(BLSH_ENOMEM, "spill buffers");
  b->spill_cap = cap;
  return BLSH_OK;
}

template <int KC>
static void launch_phase1_srp(const BatchBlock *blk, int ts, int grid1, hipStream_t s) {
  if (ts == 128) hipLaunchKernelGGL((k_batch_phase1<BLSH_COSINE, KC, 2>), dim3(grid1), dim3(kBBlock), 0, s, blk);
  else if (ts == 512) hipLaunchKernelGGL((k_batch_phase1<BLSH_COSINE, KC, 8>), dim3(grid1), dim3(kBBlock), 0, s, blk);
  else hipLaunchKernelGGL((k_batch_phase1<BLSH_COSINE, KC, 4>), dim3(grid1), dim3(kBBlock), 0, s, blk);
}

template <int KJ>
static void launch_phase1_mh(const BatchBlock *blk, int tm, int grid1, hipStream_t s) {
  if (tm == 128) hipLaunchKernelGGL((k_batch_phase1<BLSH_JACCARD, KJ, 2>), dim3(grid1), dim3(kBBlock), 0, s, blk);
  else hipLaunchKernelGGL((k_batch_phase1<BLSH_JACCARD, KJ, 1>), dim3(grid1), dim3(kBBlock), 0, s, blk);
}

template <int KJ, int KC>
static void launch_batch_kernels(BatchState *b, const BatchState::GraphKey &gk, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(kSlices), 0, s, b->d_block);
  if (gk.mode == 1) {
    hipLaunchKernelGGL((k_batch_exhaustive<KJ, KC>), dim3(gk.grid1), dim3(kBBlock), 0, s, b->d_block);
  } else {
    launch_phase1_srp<KC>(b->d_block, gk.ts, gk.grid1, s);
    launch_phase1_mh<KJ>(b->d_block, gk.tm, gk.grid1, s);
    hipLaunchKernelGGL((k_batch_phase2<KJ, KC>), dim3(gk.grid2), dim3(kBBlock), 0, s, b->d_block);
  }
  hipLaunchKernelGGL(k_batch_flush, dim3(kSlices), dim3(kBBlock), 0, s, b->d_block);
}

template <int KJ>
static void launch_batch_kernels_kc(BatchState *b, const BatchState::GraphKey &gk, hipStream_t s) {
  if (gk.kc == 16) launch_batch_kernels<KJ, 16>(b, gk, s);
  else if (gk.kc == 32) launch_batch_kernels<KJ, 32>(b, gk, s);
  else launch_batch_kernels<KJ, 64>(b, gk, s);
}

static int get_graph(BatchState *b, const BatchState::GraphKey &key, hipGraphExec_t *out) {
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) { *out = it->second; return BLSH_OK; }
  hipGraph_t g;
  BLSH_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  if (key.kj == 16) launch_batch_kernels_kc<16>(b, key, b->cap_stream);
  else if (key.kj == 32) launch_batch_kernels_kc<32>(b, key, b->cap_stream);
  else launch_batch_kernels_kc<64>(b, key, b->cap_stream);
  BLSH_HIP(hipStreamEndCapture(b->cap_stream, &g));
  hipGraphExec_t ex;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(BLSH_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  b->graphs[key] = ex;
  *out = ex;
  return BLSH_OK;
}

int verify_batched(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand, int64_t n_cand,
                   const blsh_sigs *jac, const blsh_sigs *cos, double eps, double delta, double gamma,
                   blsh_prior prior, int32_t kj, int32_t kc, blsh_result *res, int32_t *k_used, hipStream_t s,
                   int (*check_sigs_fn)(const blsh_sigs *, int, int *, int *), int mode) {
  BatchState *b = nullptr;
  int rc = batch_state(ctx, &b);
  if (rc) return rc;
  // --- tables per (measure, t); each measure has its own k ---
  const int k_given[2] = {kj, kc};
  int n_max[2] = {0, 0}, row_words[2] = {0, 0};
  const blsh_sigs *sv[2] = {jac, cos};
  bool need[2] = {false, false};
  for (int64_t i = 0; i < n_lists; ++i) need[lists[i].measure == BLSH_COSINE] = true;
  for (int me = 0; me < 2; ++me) {
    if (!need[me]) continue;
    if (!sv[me]) return fail(BLSH_EINVAL, "a list needs %s signatures", me ? "cosine" : "Jaccard");
    if (sv[me]->measure != me) return fail(BLSH_EINVAL, "signature set has the wrong measure");
    const std::vector<int> ks = k_given[me] ? std::vector<int>{k_given[me]} : std::vector<int>{16, 32, 64};
    for (int kk : ks)
      if ((rc = check_sigs_fn(sv[me], kk, &n_max[me], &row_words[me]))) return rc;
  }
  std::vector<double> ts;
  for (int64_t i = 0; i < n_lists; ++i) ts.push_back(lists[i].t);
  std::sort(ts.begin(), ts.end());
  ts.erase(std::unique(ts.begin(), ts.end()), ts.end());
  if (2 * ts.size() > size_t(kMaxBatchTables)) return fail(BLSH_EINVAL, "at most %d distinct thresholds per batch", kMaxBatchTables / 2);
  // --- work decomposition (does not depend on k) ---
  if ((rc = grow_lists(b, n_lists))) return rc;
  if (b->staged_valid) BLSH_HIP(hipEventSynchronize(b->staged));   // previous call's staging copies are done
  // list descriptors; the tile prefix sums depend on the tile shapes and are
  // built by prepare()
  const int n_slices = mode ? 1 : 2 * kXcds;
  for (int64_t i = 0; i < n_lists; ++i) {
    const blsh_list_desc &d = lists[i];
    BatchList &bl = b->h_lists[i];
    bl.offset = d.offset;
    bl.length = d.length;
    bl.query = d.query;
    bl.measure = d.measure;
    bl.table = int32_t(std::lower_bound(ts.begin(), ts.end(), d.t) - ts.begin()) * 2 + (d.measure == BLSH_COSINE);
    bl.pad = 0;
  }
  // tile prefix sums for SRP / minhash tiles of srp_tile / mh_tile candidates:
  // one array (comparator) or one per (measure, XCD slice)
  int64_t tiles = 0;
  auto build_prefix = [&](int64_t srp_tile, int64_t mh_tile) {
    tiles = 0;
    for (int x = 0; x < n_slices; ++x) b->h_prefix[int64_t(x) * (n_lists + 1)] = 0;
    for (int64_t i = 0; i < n_lists; ++i) {
      const blsh_list_desc &d = lists[i];
      const int64_t tsz = d.measure == BLSH_COSINE ? srp_tile : mh_tile;
      const int64_t nt = (d.length + tsz - 1) / tsz;
      tiles += nt;
      for (int x = 0; x < n_slices; ++x) {
        int64_t *px = b->h_prefix + int64_t(x) * (n_lists + 1);
        if (mode) {
          px[i + 1] = px[i] + nt;
        } else {
          const int me = x / kXcds, xs = x % kXcds;
          px[i + 1] = px[i] + (me == d.measure ? (int64_t(xs + 1) * nt) / kXcds - (int64_t(xs) * nt) / kXcds : 0);
        }
      }
    }
  };
  int64_t prefix_shape[2] = {-1, -1};   // tile shapes of the prefix sums last uploaded in this call
  const int64_t spill_cap = ctx->tuning.batch_spill_cap > 0
                                ? int64_t(ctx->tuning.batch_spill_cap)
                                : std::max<int64_t>(1024, std::min<int64_t>(n_cand, int64_t(1) << 24));
  if ((rc = grow_spill(b, spill_cap))) return rc;

  auto prepare = [&](int kkj, int kkc, int64_t srp_tile, int64_t mh_tile, int inreg, int grid1) -> int {
    const int kk[2] = {kkj, kkc};
    // the pinned staging (block, prefix sums) is read by the copies enqueued by
    // the previous prepare (the autotuner enqueues several per call): wait for
    // those copies before rewriting it
    BLSH_HIP(hipEventSynchronize(b->staged));
    if (prefix_shape[0] != srp_tile || prefix_shape[1] != mh_tile) {
      build_prefix(srp_tile, mh_tile);
      BLSH_HIP(hipMemcpyAsync(b->d_prefix, b->h_prefix, n_slices * (n_lists + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
      prefix_shape[0] = srp_tile;
      prefix_shape[1] = mh_tile;
    }
    BatchBlock &B = *b->h_block;
    std::memset(&B, 0, sizeof(B));
    B.lists = b->d_lists;
    B.tile_prefix = b->d_prefix;
    B.n_lists = n_lists;
    B.n_tiles = tiles;
    B.cand = cand;
    for (int me = 0; me < 2; ++me) {
      if (!need[me]) continue;
      const blsh_sigs &g = *sv[me];
      const bool om_rows = g.layout == BLSH_OBJECT_MAJOR && row_words[me] % 4 == 0 && (uintptr_t(g.data) & 15) == 0;
      const uint32_t *pfx = me == BLSH_COSINE ? (g.prefix ? g.prefix : (om_rows ? g.data : nullptr)) : nullptr;
      B.sig[me] = SigView{g.data, g.n_obj, row_words[me], g.layout == BLSH_WORD_MAJOR ? 1 : 0, pfx,
                          g.prefix ? 4 : int64_t(row_words[me])};
    }
    for (size_t ti = 0; ti < ts.size(); ++ti)
      for (int me = 0; me < 2; ++me) {
        if (!need[me]) continue;
        const int L = n_max[me] / kk[me];
        TableKey key{me, ts[ti], eps, delta, gamma, me ? 1.0 : prior.alpha, me ? 1.0 : prior.beta, kk[me], L, 0};
        const uint32_t *dt = nullptr;
        int r2 = get_table(ctx, key, nullptr, &dt, s);
        if (r2) return r2;
        B.tables[ti * 2 + me] = dt;
        B.n_levels[ti * 2 + me] = L;
      }
    B.alpha = prior.alpha;
    B.beta = prior.beta;
    B.code = res->code;
    B.acc_idx = res->acc_idx;
    B.acc_val = res->acc_val;
    B.acc_cap = res->acc_capacity;
    B.n_acc = res->n_accepted;
    B.m_dbg = res->m_debug;
    B.status = ctx->d_status;
    B.acc_cnt = b->d_stage_cnt;
    B.acc_total = b->d_stage_cnt + size_t(kSlices) * kCntStride;
    B.st_idx = b->d_st_idx;
    B.st_val = b->d_st_val;
    B.st_cap = ctx->tuning.acc_stage_cap > 0
                   ? std::min<int64_t>(kBatchStage, std::max<int64_t>(1, ctx->tuning.acc_stage_cap / kSlices))
                   : kBatchStage;
    B.spill[0] = b->d_spill[0];
    B.spill[1] = b->d_spill[1];
    B.spill_waves = grid1 * (kBBlock / kWave);
    B.spill_region = spill_cap / B.spill_waves;
    B.spill_count[0] = b->d_spill_count;
    B.spill_count[1] = b->d_spill_count + B.spill_waves;
    B.inreg_levels = inreg;
    BLSH_HIP(hipMemcpyAsync(b->d_block, b->h_block, sizeof(BatchBlock), hipMemcpyHostToDevice, s));
    // the pinned staging may be rewritten by the next call once these copies ran
    BLSH_HIP(hipEventRecord(b->staged, s));
    return BLSH_OK;
  };
  BLSH_HIP(hipMemcpyAsync(b->d_lists, b->h_lists, n_lists * sizeof(BatchList), hipMemcpyHostToDevice, s));

  auto run = [&](const BatchState::Choice &c) -> int {
    const int grid1 = std::max(kXcds, ctx->n_cu * c.bpc);   // phase 1 needs a block on every XCD slice
    int r2 = grow_spill_counts(b, int64_t(grid1) * (kBBlock / kWave));
    if (r2) return r2;
    const int ts = mode ? kExSrpTile : c.ts, tm = mode ? kExMhTile : c.tm;
    if ((r2 = prepare(c.kj, c.kc, ts, tm, c.inreg, grid1))) return r2;
    const int grid2 = std::max(1, ctx->n_cu * 4);
    hipGraphExec_t ex;
    if ((r2 = get_graph(b, BatchState::GraphKey{mode, c.kj, c.kc, ts, tm, grid1, grid2}, &ex))) return r2;
    LaunchScope ls(ctx, s, mode ? "batched_exhaustive_graph" : "batched_graph");
    BLSH_HIP(hipGraphLaunch(ex, s));
    return BLSH_OK;
  };

  // k of a measure no list uses is irrelevant: 32
  BatchState::Choice ch{kj ? kj : 32, kc ? kc : 32, kSrpTileDefault, kMhTileDefault, 2, 8};
  const int fixed_tile[2] = {ctx->tuning.batch_mh_tile, ctx->tuning.batch_srp_tile};
  if (fixed_tile[0] > 0) ch.tm = fixed_tile[0];
  if (fixed_tile[1] > 0) ch.ts = fixed_tile[1];
  if ((kj == 0 || kc == 0) && mode == 0) {
    // autotune (cached per context and batch shape): each free k in turn with
    // the other fixed (the two measures' tiles share the grid but not their
    // work), then each used measure's tile shape at its k, then in-register
    // levels x blocks per CU at the chosen shapes
    std::vector<int64_t> key{n_lists, n_cand >> 16, int64_t(need[0]), int64_t(need[1]), n_max[0], n_max[1],
                             int64_t(ts.size()), kj, kc, fixed_tile[0], fixed_tile[1]};
    auto it = b->tuned.find(key);
    if (it != b->tuned.end()) {
      ch = it->second;
    } else {
      struct EventPair {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~EventPair() {
          for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
        }
      } ev;
      BLSH_HIP(hipEventCreate(&ev.e[0]));
      BLSH_HIP(hipEventCreate(&ev.e[1]));
      hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
      auto time_of = [&](const BatchState::Choice &c, float *ms) -> int {
        int r2 = run(c);                                   // warm (tables, graph)
        if (r2) return r2;
        BLSH_HIP(hipEventRecord(e0, s));
        if ((r2 = run(c))) return r2;
        BLSH_HIP(hipEventRecord(e1, s));
        BLSH_HIP(hipEventSynchronize(e1));
        BLSH_HIP(hipEventElapsedTime(ms, e0, e1));
        return BLSH_OK;
      };
      for (int me = 0; me < 2; ++me) {
        if (k_given[me] || !need[me]) continue;
        float best = 1e30f;
        BatchState::Choice pick = ch;
        for (int kk : {16, 32, 64}) {
          BatchState::Choice c = ch;
          (me ? c.kc : c.kj) = kk;
          float ms = 0.f;
          if ((rc = time_of(c, &ms))) return rc;
          if (ms < best) { best = ms; pick = c; }
        }
        ch = pick;
      }
      for (int me = 0; me < 2; ++me) {
        if (!need[me] || fixed_tile[me] > 0) continue;
        static constexpr int kSrpShapes[] = {128, 256, 512}, kMhShapes[] = {64, 128};
        const int *shapes = me ? kSrpShapes : kMhShapes;
        const int n_shapes = me ? 3 : 2;
        float best = 1e30f;
        BatchState::Choice pick = ch;
        for (int i = 0; i < n_shapes; ++i) {
          BatchState::Choice c = ch;
          (me ? c.ts : c.tm) = shapes[i];
          float ms = 0.f;
          if ((rc = time_of(c, &ms))) return rc;
          if (ms < best) { best = ms; pick = c; }
        }
        ch = pick;
      }
      float best = 1e30f;
      BatchState::Choice pick = ch;
      for (int inreg : {1, 2, 4, kMaxLevels})   // kMaxLevels: every level in registers, no queue
        for (int bpc : {2, 4, 8}) {
          BatchState::Choice c = ch;
          c.inreg = inreg;
          c.bpc = bpc;
          float ms = 0.f;
          if ((rc = time_of(c, &ms))) return rc;
          if (ms < best) { best = ms; pick = c; }
        }
      ch = pick;
      b->tuned[key] = ch;
    }
  }
  if (ctx->tuning.batch_inreg > 0) ch.inreg = ctx->tuning.batch_inreg;
  if (ctx->tuning.batch_blocks_per_cu > 0) ch.bpc = ctx->tuning.batch_blocks_per_cu;
  if (fixed_tile[0] > 0) ch.tm = fixed_tile[0];
  if (fixed_tile[1] > 0) ch.ts = fixed_tile[1];
  if ((rc = run(ch))) return rc;
  if (k_used) { k_used[0] = ch.kj; k_used[1] = ch.kc; }
  ctx->tuning.last_batch_k_jaccard = ch.kj;
  ctx->tuning.last_batch_k_cosine = ch.kc;
  ctx->tuning.last_batch_inreg = ch.inreg;
  ctx->tuning.last_batch_blocks_per_cu = ch.bpc;
  ctx->tuning.last_batch_srp_tile = mode ? kExSrpTile : ch.ts;
  ctx->tuning.last_batch_mh_tile = mode ? kExMhTile : ch.tm;
  return BLSH_OK;
}

}  // namespace blsh
