// Batched verification of many query lists of uneven lengths in one
// graph-launched pair of persistent kernels (Algorithm 1 per candidate).
//
// Phase 1 (k_batch_phase1): persistent blocks pull tiles from a device work
//   counter.  A tile is 1024 consecutive candidates of one SRP list (one lane
//   per 4 candidates) or 256 of one minhash list (a group of k/4 lanes per
//   candidate, lane l of a wave owning candidate l).  The query's words are
//   loaded once per tile.  Each list carries its own measure and threshold,
//   hence its own decision table.  A candidate still undecided after
//   `inreg_levels` levels is spilled to a per-measure survivor queue
//   (wavefront ballot compaction); when the queue is full it simply continues
//   in registers.
// Phase 2 (k_batch_phase2): persistent blocks drain the survivor queues with
//   every lane busy: one lane per SRP survivor, one group of k/4 lanes per
//   minhash survivor, running the remaining levels.
//
// Both kernels read all their arguments from one device-resident BatchBlock,
// so the graph that holds [reset, phase 1, phase 2] is captured once per
// (k, grid) and replayed for any batch: each call only refreshes the block.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <set>

#include "device_common.h"

namespace blsh {

constexpr int kMaxBatchTables = 64;
constexpr int kSrpTile = 1024;     // candidates per SRP tile (256 lanes x 4)
constexpr int kMhTile = 256;       // candidates per minhash tile (one per lane)
constexpr int kBBlock = 256;

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
};

struct BatchBlock {
  const BatchList *lists;
  const int64_t *tile_prefix;   // [n_lists + 1]
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
  unsigned long long *counters; // [0] tile counter, [1] spill count Jaccard, [2] spill count cosine
  uint4 *spill[2];
  int64_t spill_cap;
  int32_t inreg_levels;
};

// Spill entry: x = candidate position (low), y = candidate position (high),
// z = list index, w = m | level << 16 (level = next level to run).
__device__ inline uint4 spill_entry(int64_t pos, uint32_t list, uint32_t m, uint32_t next_level) {
  return make_uint4(uint32_t(pos), uint32_t(uint64_t(pos) >> 32), list, m | (next_level << 16));
}

__device__ inline void emit_block(const BatchBlock &B, bool pred, int64_t idx, float val) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd((unsigned long long *)B.n_acc, (unsigned long long)__popcll(mask));
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

// Reserve spill slots for the lanes with `pred`; returns whether this lane got one.
__device__ inline bool spill_push(const BatchBlock &B, int meas, bool pred, uint4 e) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return false;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(&B.counters[1 + meas], (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  if (!pred) return false;
  const unsigned long long pos = base + lanes_below(mask);
  if (int64_t(pos) >= B.spill_cap) return false;
  B.spill[meas][pos] = e;
  return true;
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
// phase 1: tiles
// ---------------------------------------------------------------------------
template <int K>
__device__ void srp_tile(const BatchBlock &B, const BatchList &Ls, int32_t list_id, int64_t tile_in_list,
                         const int *s_min, const uint32_t *tab, int L) {
  const SigView &S = B.sig[BLSH_COSINE];
  const int words = int(tab[2]);
  const int64_t base = Ls.offset + tile_in_list * kSrpTile;
  const int64_t end = Ls.offset + Ls.length;
  const int64_t c0 = base + int64_t(threadIdx.x) * 4;
  const uint32_t q = Ls.query;
  const bool q_ok = q < S.n_obj;
  uint32_t y[4] = {0, 0, 0, 0};
  uint32_t alive = 0, bad = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (c0 + p < end) {
      y[p] = __builtin_nontemporal_load(B.cand + c0 + p);
      if (q_ok && y[p] < S.n_obj) alive |= 1u << p; else bad |= 1u << p;
    }
  }
  uint32_t m[4] = {0, 0, 0, 0};
  uint8_t code[4] = {0, 0, 0, 0};
  uint32_t emit = 0;
  const int J = min(L, B.inreg_levels);
  int j = 0;
  for (; j < J && alive; ++j) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
      if (alive & (1u << p)) m[p] += srp_level_word_agree<K>(S, q, y[p], j);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (!(alive & (1u << p))) continue;
      if (int(m[p]) < s_min[j]) { code[p] = uint8_t((BLSH_PRUNED << 6) | j); alive &= ~(1u << p); }
      else if (accept_bit(tab, words, j, int(m[p]))) { code[p] = uint8_t((BLSH_ACCEPT_CONC << 6) | j); alive &= ~(1u << p); emit |= 1u << p; }
      else if (j == L - 1) { code[p] = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); alive &= ~(1u << p); emit |= 1u << p; }
    }
  }
  // spill what is still undecided; what cannot be spilled continues here
  uint32_t kept = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const bool want = (alive >> p) & 1u;
    const bool ok = spill_push(B, BLSH_COSINE, want, spill_entry(c0 + p, uint32_t(list_id), m[p], uint32_t(J)));
    if (want && !ok) kept |= 1u << p;
  }
  alive = kept;
  for (j = J; j < L && alive; ++j) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
      if (alive & (1u << p)) m[p] += srp_level_word_agree<K>(S, q, y[p], j);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      if (!(alive & (1u << p))) continue;
      if (int(m[p]) < s_min[j]) { code[p] = uint8_t((BLSH_PRUNED << 6) | j); alive &= ~(1u << p); }
      else if (accept_bit(tab, words, j, int(m[p]))) { code[p] = uint8_t((BLSH_ACCEPT_CONC << 6) | j); alive &= ~(1u << p); emit |= 1u << p; }
      else if (j == L - 1) { code[p] = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); alive &= ~(1u << p); emit |= 1u << p; }
    }
  }
  if (bad) raise_status(B.status, BLSH_EBADID);
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (c0 + p >= end) continue;
    B.code[c0 + p] = (bad >> p) & 1u ? uint8_t(0xFF) : code[p];
    if (B.m_dbg) B.m_dbg[c0 + p] = uint16_t(m[p]);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const bool e = (emit >> p) & 1u;
    const float v = e ? map_estimate(BLSH_COSINE, int(m[p]), ((code[p] & 63) + 1) * K, 1.0, 1.0) : 0.f;
    emit_block(B, e, c0 + p, v);
  }
}

template <int G, int S>
struct BatchMhStep {
  template <int K>
  __device__ static inline void run(const SigView &sv, uint4 hq, uint32_t y, uint32_t alive, int j, int r,
                                    uint32_t &own) {
    const uint32_t ys = group_bcast<G, S>(y);
    const uint32_t al = group_bcast<G, S>(alive);
    uint32_t c = 0;
    if (al) {
      const uint4 hy = *reinterpret_cast<const uint4 *>(sv.data + size_t(ys) * sv.row_words + j * K + 4 * r);
      c = uint32_t(hq.x == hy.x) + uint32_t(hq.y == hy.y) + uint32_t(hq.z == hy.z) + uint32_t(hq.w == hy.w);
    }
    c = group_sum<G>(c);
    if (r == S) own = c;
    if constexpr (S + 1 < G) BatchMhStep<G, S + 1>::template run<K>(sv, hq, y, alive, j, r, own);
  }
};

template <int K>
__device__ void minhash_tile(const BatchBlock &B, const BatchList &Ls, int32_t list_id, int64_t tile_in_list,
                             const int *s_min, const uint32_t *tab, int L) {
  constexpr int G = K / 4;
  const SigView &S = B.sig[BLSH_JACCARD];
  const int words = int(tab[2]);
  const int64_t end = Ls.offset + Ls.length;
  const int64_t c = Ls.offset + tile_in_list * kMhTile + threadIdx.x;
  const int lane = lane_id(), r = lane & (G - 1);
  const uint32_t q = Ls.query;
  const bool q_ok = q < S.n_obj;
  uint32_t y = 0, alive = 0;
  bool bad = false;
  if (c < end) {
    y = __builtin_nontemporal_load(B.cand + c);
    if (q_ok && y < S.n_obj) alive = 1; else { bad = true; y = 0; }
  }
  uint32_t m = 0;
  uint8_t code = 0;
  bool emit = false;
  const int J = min(L, B.inreg_levels);
  auto level = [&](int j) {
    uint4 hq = make_uint4(0, 0, 0, 0);
    if (q_ok) hq = *reinterpret_cast<const uint4 *>(S.data + size_t(q) * S.row_words + j * K + 4 * r);
    uint32_t own = 0;
    BatchMhStep<G, 0>::template run<K>(S, hq, y, alive, j, r, own);
    if (alive) {
      m += own;
      if (int(m) < s_min[j]) { code = uint8_t((BLSH_PRUNED << 6) | j); alive = 0; }
      else if (accept_bit(tab, words, j, int(m))) { code = uint8_t((BLSH_ACCEPT_CONC << 6) | j); alive = 0; emit = true; }
      else if (j == L - 1) { code = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); alive = 0; emit = true; }
    }
  };
  for (int j = 0; j < J; ++j) {
    if (__ballot(alive != 0) == 0) break;
    level(j);
  }
  const bool want = alive != 0;
  const bool ok = spill_push(B, BLSH_JACCARD, want, spill_entry(c, uint32_t(list_id), m, uint32_t(J)));
  if (ok) alive = 0;
  for (int j = J; j < L; ++j) {
    if (__ballot(alive != 0) == 0) break;
    level(j);
  }
  if (bad) raise_status(B.status, BLSH_EBADID);
  if (c < end) {
    B.code[c] = bad ? uint8_t(0xFF) : code;
    if (B.m_dbg) B.m_dbg[c] = uint16_t(m);
  }
  const float v = emit ? map_estimate(BLSH_JACCARD, int(m), ((code & 63) + 1) * K, B.alpha, B.beta) : 0.f;
  emit_block(B, emit, c, v);
}

__device__ inline int64_t list_of_tile(const int64_t *prefix, int64_t n_lists, int64_t t) {
  int64_t lo = 0, hi = n_lists - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int K>
__global__ __launch_bounds__(kBBlock) void k_batch_phase1(const BatchBlock *__restrict__ Bp) {
  const BatchBlock &B = *Bp;
  __shared__ int s_min[kMaxLevels];
  __shared__ long long s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (long long)atomicAdd(&B.counters[0], 1ull);
    __syncthreads();
    const long long t = s_tile;
    if (t >= B.n_tiles) break;
    const int64_t l = list_of_tile(B.tile_prefix, B.n_lists, t);
    const BatchList Ls = B.lists[l];
    const uint32_t *tab = B.tables[Ls.table];
    const int L = B.n_levels[Ls.table];
    if (threadIdx.x < kMaxLevels) s_min[threadIdx.x] = int(threadIdx.x) < L ? int(tab[kTabMinOff + threadIdx.x]) : 0x7fffffff;
    __syncthreads();
    if (Ls.measure == BLSH_COSINE) srp_tile<K>(B, Ls, int32_t(l), t - B.tile_prefix[l], s_min, tab, L);
    else minhash_tile<K>(B, Ls, int32_t(l), t - B.tile_prefix[l], s_min, tab, L);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// phase 2: spilled survivors
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(kBBlock) void k_batch_phase2(const BatchBlock *__restrict__ Bp) {
  constexpr int G = K / 4;
  const BatchBlock &B = *Bp;
  const int lane = lane_id();
  // SRP survivors: one lane each
  {
    const int64_t n = min<int64_t>(int64_t(B.counters[1 + BLSH_COSINE]), B.spill_cap);
    const SigView &S = B.sig[BLSH_COSINE];
    const int64_t stride = int64_t(gridDim.x) * kBBlock;
    for (int64_t i0 = int64_t(blockIdx.x) * kBBlock; i0 < n; i0 += stride) {
      const int64_t i = i0 + threadIdx.x;
      bool act = i < n;
      int64_t pos = 0;
      uint32_t m = 0, q = 0, yv = 0;
      int j = 0, L = 0, words = 0;
      const uint32_t *tab = nullptr;
      uint8_t code = 0;
      bool emit = false;
      if (act) {
        const uint4 e = B.spill[BLSH_COSINE][i];
        pos = int64_t(uint64_t(e.x) | (uint64_t(e.y) << 32));
        const BatchList Ls = B.lists[e.z];
        tab = B.tables[Ls.table];
        L = B.n_levels[Ls.table];
        words = int(tab[2]);
        m = e.w & 0xFFFFu;
        j = int(e.w >> 16);
        q = Ls.query;
        yv = B.cand[pos];
        for (; j < L; ++j) {
          m += srp_level_word_agree<K>(S, q, yv, j);
          if (int(m) < int(tab[kTabMinOff + j])) { code = uint8_t((BLSH_PRUNED << 6) | j); break; }
          if (accept_bit(tab, words, j, int(m))) { code = uint8_t((BLSH_ACCEPT_CONC << 6) | j); emit = true; break; }
          if (j == L - 1) { code = uint8_t((BLSH_ACCEPT_NMAX << 6) | j); emit = true; break; }
        }
        B.code[pos] = code;
        if (B.m_dbg) B.m_dbg[pos] = uint16_t(m);
      }
      const float v = emit ? map_estimate(BLSH_COSINE, int(m), ((code & 63) + 1) * K, 1.0, 1.0) : 0.f;
      emit_block(B, emit, pos, v);
    }
  }
  // minhash survivors: one group of G lanes each
  {
    const int64_t n = min<int64_t>(int64_t(B.counters[1 + BLSH_JACCARD]), B.spill_cap);
    const SigView &S = B.sig[BLSH_JACCARD];
    constexpr int PER_BLOCK = kBBlock / G;
    const int g = threadIdx.x / G, r = threadIdx.x % G;
    const int64_t stride = int64_t(gridDim.x) * PER_BLOCK;
    for (int64_t i0 = int64_t(blockIdx.x) * PER_BLOCK; i0 < n; i0 += stride) {
      const int64_t i = i0 + g;
      const bool act = i < n;
      int64_t pos = 0;
      uint32_t m = 0, q = 0, yv = 0;
      int j = 0, L = 0, words = 0;
      const uint32_t *tab = nullptr;
      if (act) {
        const uint4 e = B.spill[BLSH_JACCARD][i];
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
          const uint4 hq = *reinterpret_cast<const uint4 *>(S.data + size_t(q) * S.row_words + j * K + 4 * r);
          const uint4 hy = *reinterpret_cast<const uint4 *>(S.data + size_t(yv) * S.row_words + j * K + 4 * r);
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
      const float v = e ? map_estimate(BLSH_JACCARD, int(m), ((code & 63) + 1) * K, B.alpha, B.beta) : 0.f;
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
  const int64_t t0 = Ls.offset + tile_in_list * kSrpTile;
  for (int64_t c0 = t0; c0 < min(end, t0 + kSrpTile); c0 += PER_BLOCK) {
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
  const int64_t t0 = Ls.offset + tile_in_list * kMhTile;
  for (int64_t c0 = t0; c0 < min(end, t0 + kMhTile); c0 += PER_BLOCK) {
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

template <int K>
__global__ __launch_bounds__(kBBlock) void k_batch_exhaustive(const BatchBlock *__restrict__ Bp) {
  const BatchBlock &B = *Bp;
  __shared__ long long s_tile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (long long)atomicAdd(&B.counters[0], 1ull);
    __syncthreads();
    const long long t = s_tile;
    if (t >= B.n_tiles) break;
    const int64_t l = list_of_tile(B.tile_prefix, B.n_lists, t);
    const BatchList Ls = B.lists[l];
    const uint32_t *tab = B.tables[Ls.table];
    const int L = B.n_levels[Ls.table];
    const int64_t tl = t - B.tile_prefix[l];
    if (Ls.measure == BLSH_COSINE) {
      const int W = L * K / 32;   // words compared: n_max bits
      if (W == 4) srp_tile_exhaustive<K, 1>(B, Ls, tl, tab, L);
      else if (W == 8) srp_tile_exhaustive<K, 2>(B, Ls, tl, tab, L);
      else if (W == 16) srp_tile_exhaustive<K, 4>(B, Ls, tl, tab, L);
      else if (W == 32) srp_tile_exhaustive<K, 8>(B, Ls, tl, tab, L);
      else srp_tile_exhaustive<K, 16>(B, Ls, tl, tab, L);
    } else {
      minhash_tile_exhaustive<K>(B, Ls, tl, tab, L, L * K);
    }
    __syncthreads();
  }
}

__global__ void k_batch_reset(const BatchBlock *__restrict__ Bp) {
  const BatchBlock &B = *Bp;
  if (threadIdx.x < 3) B.counters[threadIdx.x] = 0;
  if (threadIdx.x == 3) *B.n_acc = 0;
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
  unsigned long long *d_counters = nullptr;
  uint4 *d_spill[2] = {nullptr, nullptr};
  int64_t spill_cap = 0;
  hipEvent_t staged{};
  bool staged_valid = false;
  hipStream_t cap_stream{};
  struct GraphKey {
    int mode, k, grid1, grid2;
    bool operator<(const GraphKey &o) const {
      return std::tie(mode, k, grid1, grid2) < std::tie(o.mode, o.k, o.grid1, o.grid2);
    }
  };
  std::map<GraphKey, hipGraphExec_t> graphs;
  struct Choice { int k, inreg, bpc; };
  std::map<std::vector<int64_t>, Choice> tuned;
};

static void batch_free(BatchState *b) {
  if (!b) return;
  for (auto &g : b->graphs) hipGraphExecDestroy(g.second);
  if (b->d_block) hipFree(b->d_block);
  if (b->h_block) hipHostFree(b->h_block);
  if (b->d_lists) hipFree(b->d_lists);
  if (b->h_lists) hipHostFree(b->h_lists);
  if (b->d_prefix) hipFree(b->d_prefix);
  if (b->h_prefix) hipHostFree(b->h_prefix);
  if (b->d_counters) hipFree(b->d_counters);
  for (auto *p : b->d_spill) if (p) hipFree(p);
  if (b->staged_valid) hipEventDestroy(b->staged);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  delete b;
}

void batch_state_free(void *p) { batch_free(static_cast<BatchState *>(p)); }

static int batch_state(blsh_ctx *ctx, BatchState **out) {
  if (!ctx->batch) {
    auto *b = new (std::nothrow) BatchState();
    if (!b) return fail(BLSH_ENOMEM, "host allocation failed");
    if (hipMalloc(&b->d_block, sizeof(BatchBlock)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&b->h_block), sizeof(BatchBlock), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&b->d_counters, 256) != hipSuccess ||
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
  if (b->d_lists) hipFree(b->d_lists);
  if (b->h_lists) hipHostFree(b->h_lists);
  if (b->d_prefix) hipFree(b->d_prefix);
  if (b->h_prefix) hipHostFree(b->h_prefix);
  b->d_lists = b->h_lists = nullptr;
  b->d_prefix = b->h_prefix = nullptr;
  b->lists_cap = 0;
  const int64_t cap = std::max<int64_t>(n_lists, 1024);
  if (hipMalloc(&b->d_lists, cap * sizeof(BatchList)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&b->h_lists), cap * sizeof(BatchList), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&b->d_prefix, (cap + 1) * sizeof(int64_t)) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&b->h_prefix), (cap + 1) * sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
    return fail(BLSH_ENOMEM, "list buffers");
  b->lists_cap = cap;
  return BLSH_OK;
}

static int grow_spill(BatchState *b, int64_t cap) {
  if (b->spill_cap >= cap) return BLSH_OK;
  BLSH_HIP(hipDeviceSynchronize());
  for (auto *&p : b->d_spill) { if (p) hipFree(p); p = nullptr; }
  b->spill_cap = 0;
  for (auto *&p : b->d_spill)
    if (hipMalloc(&p, size_t(cap) * sizeof(uint4)) != hipSuccess) return fail(BLSH_ENOMEM, "spill buffers");
  b->spill_cap = cap;
  return BLSH_OK;
}

template <int K>
static void launch_batch_kernels(BatchState *b, int mode, int grid1, int grid2, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, b->d_block);
  if (mode == 1) {
    hipLaunchKernelGGL(k_batch_exhaustive<K>, dim3(grid1), dim3(kBBlock), 0, s, b->d_block);
    return;
  }
  hipLaunchKernelGGL(k_batch_phase1<K>, dim3(grid1), dim3(kBBlock), 0, s, b->d_block);
  hipLaunchKernelGGL(k_batch_phase2<K>, dim3(grid2), dim3(kBBlock), 0, s, b->d_block);
}

static int get_graph(BatchState *b, int mode, int k, int grid1, int grid2, hipGraphExec_t *out) {
  BatchState::GraphKey key{mode, k, grid1, grid2};
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) { *out = it->second; return BLSH_OK; }
  hipGraph_t g;
  BLSH_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  if (k == 16) launch_batch_kernels<16>(b, mode, grid1, grid2, b->cap_stream);
  else if (k == 32) launch_batch_kernels<32>(b, mode, grid1, grid2, b->cap_stream);
  else launch_batch_kernels<64>(b, mode, grid1, grid2, b->cap_stream);
  BLSH_HIP(hipStreamEndCapture(b->cap_stream, &g));
  hipGraphExec_t ex;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(BLSH_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  b->graphs[key] = ex;
  *out = ex;
  return BLSH_OK;
}

int verify_batched(blsh_ctx *ctx, const blsh_list_desc *lists, int64_t n_lists, const uint32_t *cand, int64_t n_cand,
                   const blsh_sigs *jac, const blsh_sigs *cos, double eps, double delta, double gamma,
                   blsh_prior prior, int32_t k, blsh_result *res, int32_t *k_used, hipStream_t s,
                   int (*check_sigs_fn)(const blsh_sigs *, int, int *, int *), int mode) {
  BatchState *b = nullptr;
  int rc = batch_state(ctx, &b);
  if (rc) return rc;
  // --- tables per (measure, t) ---
  std::vector<int> ks = k ? std::vector<int>{k} : std::vector<int>{16, 32, 64};
  int n_max[2] = {0, 0}, row_words[2] = {0, 0};
  const blsh_sigs *sv[2] = {jac, cos};
  bool need[2] = {false, false};
  for (int64_t i = 0; i < n_lists; ++i) need[lists[i].measure == BLSH_COSINE] = true;
  for (int me = 0; me < 2; ++me) {
    if (!need[me]) continue;
    if (!sv[me]) return fail(BLSH_EINVAL, "a list needs %s signatures", me ? "cosine" : "Jaccard");
    if (sv[me]->measure != me) return fail(BLSH_EINVAL, "signature set has the wrong measure");
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
  int64_t tiles = 0;
  b->h_prefix[0] = 0;
  for (int64_t i = 0; i < n_lists; ++i) {
    const blsh_list_desc &d = lists[i];
    BatchList &bl = b->h_lists[i];
    bl.offset = d.offset;
    bl.length = d.length;
    bl.query = d.query;
    bl.measure = d.measure;
    bl.table = int32_t(std::lower_bound(ts.begin(), ts.end(), d.t) - ts.begin()) * 2 + (d.measure == BLSH_COSINE);
    bl.pad = 0;
    const int64_t tsz = d.measure == BLSH_COSINE ? kSrpTile : kMhTile;
    tiles += (d.length + tsz - 1) / tsz;
    b->h_prefix[i + 1] = tiles;
  }
  const int64_t spill_cap = ctx->tuning.batch_spill_cap > 0
                                ? int64_t(ctx->tuning.batch_spill_cap)
                                : std::max<int64_t>(1024, std::min<int64_t>(n_cand, int64_t(1) << 24));
  if ((rc = grow_spill(b, spill_cap))) return rc;

  auto prepare = [&](int kk, int inreg) -> int {
    BatchBlock &B = *b->h_block;
    std::memset(&B, 0, sizeof(B));
    B.lists = b->d_lists;
    B.tile_prefix = b->d_prefix;
    B.n_lists = n_lists;
    B.n_tiles = tiles;
    B.cand = cand;
    for (int me = 0; me < 2; ++me) {
      if (!need[me]) continue;
      B.sig[me] = SigView{sv[me]->data, sv[me]->n_obj, row_words[me], sv[me]->layout == BLSH_WORD_MAJOR ? 1 : 0};
    }
    for (size_t ti = 0; ti < ts.size(); ++ti)
      for (int me = 0; me < 2; ++me) {
        if (!need[me]) continue;
        const int L = n_max[me] / kk;
        TableKey key{me, ts[ti], eps, delta, gamma, me ? 1.0 : prior.alpha, me ? 1.0 : prior.beta, kk, L, 0};
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
    B.counters = b->d_counters;
    B.spill[0] = b->d_spill[0];
    B.spill[1] = b->d_spill[1];
    B.spill_cap = spill_cap;
    B.inreg_levels = inreg;
    BLSH_HIP(hipMemcpyAsync(b->d_block, b->h_block, sizeof(BatchBlock), hipMemcpyHostToDevice, s));
    // the pinned staging may be rewritten by the next call once these copies ran
    BLSH_HIP(hipEventRecord(b->staged, s));
    return BLSH_OK;
  };
  BLSH_HIP(hipMemcpyAsync(b->d_lists, b->h_lists, n_lists * sizeof(BatchList), hipMemcpyHostToDevice, s));
  BLSH_HIP(hipMemcpyAsync(b->d_prefix, b->h_prefix, (n_lists + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));

  auto run = [&](int kk, int inreg, int bpc) -> int {
    int r2 = prepare(kk, inreg);
    if (r2) return r2;
    const int grid1 = std::max(1, ctx->n_cu * bpc);
    const int grid2 = std::max(1, ctx->n_cu * 4);
    hipGraphExec_t ex;
    if ((r2 = get_graph(b, mode, kk, grid1, grid2, &ex))) return r2;
    LaunchScope ls(ctx, s, mode ? "batched_exhaustive_graph" : "batched_graph");
    BLSH_HIP(hipGraphLaunch(ex, s));
    return BLSH_OK;
  };

  BatchState::Choice ch{k ? k : 32, 2, 4};
  if (k == 0 && mode == 0) {
    // autotune key: batch shape (the choice is cached per context)
    std::vector<int64_t> key{n_lists, n_cand >> 16, int64_t(need[0]), int64_t(need[1]), n_max[0], n_max[1],
                             int64_t(ts.size())};
    auto it = b->tuned.find(key);
    if (it != b->tuned.end()) {
      ch = it->second;
    } else {
      hipEvent_t e0, e1;
      BLSH_HIP(hipEventCreate(&e0));
      BLSH_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      for (int kk : {16, 32, 64})
        for (int inreg : {1, 2, 4})
          for (int bpc : {2, 4, 8}) {
            if ((rc = run(kk, inreg, bpc))) return rc;      // warm (tables, graph)
            BLSH_HIP(hipEventRecord(e0, s));
            if ((rc = run(kk, inreg, bpc))) return rc;
            BLSH_HIP(hipEventRecord(e1, s));
            BLSH_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            BLSH_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) { best = ms; ch = BatchState::Choice{kk, inreg, bpc}; }
          }
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      b->tuned[key] = ch;
    }
  } else {
    ch.k = k;
  }
  if (ctx->tuning.batch_inreg > 0) ch.inreg = ctx->tuning.batch_inreg;
  if (ctx->tuning.batch_blocks_per_cu > 0) ch.bpc = ctx->tuning.batch_blocks_per_cu;
  if ((rc = run(ch.k, ch.inreg, ch.bpc))) return rc;
  if (k_used) *k_used = ch.k;
  ctx->tuning.last_batch_k = ch.k;
  ctx->tuning.last_batch_inreg = ch.inreg;
  ctx->tuning.last_batch_blocks_per_cu = ch.bpc;
  return BLSH_OK;
}

}  // namespace blsh
