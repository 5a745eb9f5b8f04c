// Device helpers for the gfx950 kernels (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace blsh {

constexpr int kWave = 64;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Arguments shared by the verification kernels (passed by value).
struct VerifyArgs {
  // candidates
  int32_t kind;
  const uint32_t *x, *y;                 // PAIRS
  const uint32_t *query;                 // QUERY_LISTS
  const int64_t *offsets;
  const uint32_t *cand;
  int64_t n_lists;
  int64_t all_n;                         // ALL_PAIRS
  int64_t c_begin, c_end;                // candidate range of this launch
  // signatures
  const uint32_t *sig;
  int64_t n_obj;
  int32_t row_words;                     // object-major row length in 32-bit words
  const uint32_t *pfx;                   // hashes 0..127 of object i at pfx + i * pfx_stride (16 B), or null
  int32_t pfx_stride;
  // decision table
  const uint32_t *table;
  int32_t n_levels;                      // levels run (n_max/k, or h/k for Lite)
  int32_t measure;
  // outputs
  uint8_t *code;
  uint64_t *acc_idx;
  float *acc_val;
  int64_t acc_cap;
  int64_t *n_acc;
  uint16_t *m_dbg;
  // survivor queue: candidate index relative to c_begin (Lite survivors, and
  // SRP candidates undecided after the 128-hash prefix when q_m is set: then
  // q_m holds m | next level << 16 for the tail kernel).  kSlices slices of
  // q_cap entries; the count of slice s is q_cnt[s * kCntStride].
  uint32_t *q_rel;
  uint32_t *q_m;
  int64_t *q_cnt;
  int64_t q_cap;
  // accepted-pair staging: kSlices slices of st_cap entries (index relative to
  // c_begin, value), counts at acc_cnt[s * kCntStride], appended to the
  // caller's list by k_acc_flush; entries that find their slice full go to the
  // list directly.  Positions in the list come from the running count
  // *acc_total; the last flush of a call stores it to *n_acc.
  int64_t *acc_cnt;
  uint32_t *st_rel;
  float *st_val;
  int64_t st_cap;
  int64_t *acc_total;
  int32_t *status;
  // exact similarity (Lite): the caller's vectors
  int32_t ex_kind;
  const float *ex_dense;
  int64_t ex_dim;
  const int64_t *ex_offsets;
  const uint32_t *ex_indices;
  const float *ex_values;
  // exhaustive
  int32_t mode;                          // 0 replay, 1 replay-lite, 2 mle
  int32_t count_levels;                  // levels compared in full (n_max/k)
  double t;
  // BLSH_TILES: the launch runs tiles [t_begin, t_end) (in any order of their
  // numbering); n_cand bounds every candidate index written
  const blsh_tile *tiles;
  int64_t t_begin, t_end;
  int64_t n_cand;
  // staging values are raw (m | n << 16, as the float's bits): the flush
  // computes S_hat from them (tiles path)
  int32_t st_raw;
  // tiles path: the staging holds one region of st_cap entries per wave of the
  // persistent grid, filled in order -- the candidate index (absolute, 8 B)
  // in st_idx and the raw value in st_val; wave w leaves its count in wst_cnt[w]
  uint64_t *st_idx;
  uint32_t *wst_cnt;
  // tiles path, Lite: the staged pairs' ids (x, y) beside st_idx
  uint2 *st_xy;
  // tiles path: the signature array's size in bytes when a row's offset fits
  // 32 bits through a 24-bit multiply (n_obj <= 2^24, size < 2^32): the rows
  // are then read as a buffer with 32-bit offsets; else 0
  uint32_t sig_buf_bytes;
};

__device__ inline int lane_id() { return __lane_id(); }

// Device-scope atomics on one address (or one cache line) serialise at the
// memory side, about 12 ns apiece on MI355X; spread over counters on lines of
// their own they run concurrently.  Queue and staging counts are therefore
// split into kSlices slices, 256 bytes apart, and a wave uses the slice of its
// launch-wide wave number.
constexpr int kSlices = 256;
constexpr int kCntStride = 32;   // int64 words between slice counters (256 B)

__device__ inline int wave_slice() {
  return __builtin_amdgcn_readfirstlane(int((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kSlices - 1)));
}

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ inline void raise_status(int32_t *status, int32_t code) {
  if (status) atomicCAS(status, 0, code);
}

// Bijective remap of block ids so that each XCD (blocks are dealt round-robin
// over the 8 XCDs) processes one contiguous range of tiles.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
  const int64_t xcd = b & 7, idx = b >> 3;
  const int64_t per = nb >> 3, rem = nb & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Row-major decoding of the all-pairs index c -> (i, j), i < j < n.
__device__ inline void all_pairs_decode(int64_t c, int64_t n, uint32_t &i_out, uint32_t &j_out) {
  const double b = 2.0 * double(n) - 1.0;
  int64_t i = int64_t((b - sqrt(b * b - 8.0 * double(c))) * 0.5);
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  auto start = [n](int64_t r) { return r * n - r * (r + 1) / 2; };
  while (i > 0 && start(i) > c) --i;
  while (i < n - 2 && start(i + 1) <= c) ++i;
  i_out = uint32_t(i);
  j_out = uint32_t(c - start(i) + i + 1);
}

// List containing candidate position c: the l with offsets[l] <= c < offsets[l+1].
__device__ inline int64_t list_of(const int64_t *offsets, int64_t n_lists, int64_t c) {
  int64_t lo = 0, hi = n_lists - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline bool fetch_candidate(const VerifyArgs &a, int64_t c, uint32_t &xi, uint32_t &yi) {
  if (a.kind == BLSH_PAIRS) {
    xi = __builtin_nontemporal_load(a.x + c);
    yi = __builtin_nontemporal_load(a.y + c);
  } else if (a.kind == BLSH_ALL_PAIRS) {
    all_pairs_decode(c, a.all_n, xi, yi);
  } else {
    const int64_t l = list_of(a.offsets, a.n_lists, c);
    xi = a.query[l];
    yi = __builtin_nontemporal_load(a.cand + c);
  }
  return xi < a.n_obj && yi < a.n_obj;
}

// cos(x) for x in [0, pi/2] from its Taylor series through x^24 (truncation
// below (pi/2)^26 / 26! < 2e-21), in Horner form: a few registers, no range
// reduction.  The factors 1/((2i-1) 2i) are compile-time constants, so each
// term is one multiply and one fused multiply-add (no FP64 division).
__device__ inline double cos_quarter(double x) {
  const double x2 = x * x;
  double c = 1.0;
#pragma unroll
  for (int i = 12; i >= 1; --i) {
    constexpr double one = 1.0;
    const double inv = one / double((2 * i - 1) * (2 * i));   // folded: i is a constant after unrolling
    c = __builtin_fma(-c * x2, inv, 1.0);
  }
  return c;
}

// S_hat for an emitted pair (Section 4 eqn map; Section 4.1 Beta mode; Section 4.2 r2c(m/n)).
__device__ inline float map_estimate(int measure, int m, int n, double alpha, double beta) {
  if (measure == BLSH_JACCARD) {
    double s = (m + alpha - 1.0) / (n + alpha + beta - 2.0);
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    return float(s);
  }
  double r = double(m) / double(n);
  r = r < 0.5 ? 0.5 : r;
  return float(cos_quarter(3.14159265358979323846 * (1.0 - r)));   // r2c: cos(pi (1 - r)), r in [0.5, 1]
}

__device__ inline double tab_f64(const uint32_t *tab, int w) {
  return __hiloint2double(int(tab[w + 1]), int(tab[w]));
}

__device__ inline bool accept_bit(const uint32_t *tab, int words, int j, int m) {
  return (tab[kTabAccOff + j * words + (m >> 5)] >> (m & 31)) & 1u;
}

// Accepted list, direct: one atomic on the running count per call.
__device__ inline void emit_direct(const VerifyArgs &a, bool pred, uint64_t idx, float val) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd((unsigned long long *)a.acc_total, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  if (pred) {
    const unsigned long long pos = base + lanes_below(mask);
    if (int64_t(pos) < a.acc_cap) {
      a.acc_idx[pos] = idx;
      a.acc_val[pos] = val;
    } else {
      raise_status(a.status, BLSH_ETRUNCATED);
    }
  }
}

// Wave-level compaction of (idx, val) into the wave's staging slice (the
// caller's list for entries past the slice's capacity); called in converged
// control flow by every active lane.  c_begin: the launch's first candidate.
__device__ inline void emit_accepted_from(const VerifyArgs &a, bool pred, uint64_t idx, float val, int64_t c_begin) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  {
    const int s = wave_slice();
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader)
      base = atomicAdd((unsigned long long *)(a.acc_cnt + s * kCntStride), (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    const unsigned long long pos = base + lanes_below(mask);
    if (pred && int64_t(pos) < a.st_cap) {
      a.st_rel[size_t(s) * a.st_cap + pos] = uint32_t(idx - uint64_t(c_begin));
      a.st_val[size_t(s) * a.st_cap + pos] = val;
      pred = false;
    }
  }
  emit_direct(a, pred, idx, val);
}

__device__ inline void emit_accepted(const VerifyArgs &a, bool pred, uint64_t idx, float val) {
  emit_accepted_from(a, pred, idx, val, a.c_begin);
}

// Position of a wave's `total` new entries in its survivor-queue slice (valid
// in every lane); the queue is sized so that a slice never overflows, and an
// entry past q_cap would be dropped with BLSH_EDEVICE raised.
__device__ inline int64_t queue_reserve(const VerifyArgs &a, int s, uint32_t total, int leader) {
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd((unsigned long long *)(a.q_cnt + s * kCntStride), (unsigned long long)total);
  return int64_t(__shfl(base, leader));
}

// Wave-level compaction of Lite survivors into the exact-similarity queue
// (entries are candidate indices relative to the launch's c_begin).
__device__ inline void push_survivor(const VerifyArgs &a, bool pred, int64_t c) {
  const uint64_t mask = __ballot(pred);
  if (mask == 0) return;
  const int s = wave_slice();
  const int64_t base = queue_reserve(a, s, uint32_t(__popcll(mask)), __ffsll((unsigned long long)mask) - 1);
  if (pred) {
    const int64_t pos = base + lanes_below(mask);
    if (pos < a.q_cap) a.q_rel[size_t(s) * a.q_cap + pos] = uint32_t(c - a.c_begin);
    else raise_status(a.status, BLSH_EDEVICE);
  }
}

// Wave-level compaction of a lane's P candidates (bit p of `want`: candidate
// c0 + p, with mj[p] = m | next level << 16) into the survivor queue with one
// atomic per wave.
template <int P>
__device__ inline void push_survivors(const VerifyArgs &a, uint32_t want, int64_t c0, const uint32_t *mj) {
  uint64_t mask[P];
  uint32_t total = 0;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    mask[p] = __ballot((want >> p) & 1u);
    total += uint32_t(__popcll(mask[p]));
  }
  if (total == 0) return;
  const int s = wave_slice();
  int64_t base = queue_reserve(a, s, total, 0);
  uint32_t *rel = a.q_rel + size_t(s) * a.q_cap;
  uint32_t *qm = a.q_m + size_t(s) * a.q_cap;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if ((want >> p) & 1u) {
      const int64_t pos = base + lanes_below(mask[p]);
      if (pos < a.q_cap) {
        rel[pos] = uint32_t(c0 + p - a.c_begin);
        qm[pos] = mj[p];
      } else {
        raise_status(a.status, BLSH_EDEVICE);
      }
    }
    base += __popcll(mask[p]);
  }
}

// Order this wave's LDS writes before its later LDS reads (and vice versa).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP lane permutations (GFX9 encodings).
constexpr int kDppQuadXor1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kDppRowMirror = 0x140;   // lane i <- 15 - i within a row of 16
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within each half row

template <int CTRL>
__device__ inline uint32_t dpp(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of G lanes (G in {1,2,4,8,16}); every lane of the
// group receives the total.  All lanes of the wave must be active.
template <int G>
__device__ inline uint32_t group_sum(uint32_t v) {
  if constexpr (G >= 2) v += dpp<kDppQuadXor1>(v);
  if constexpr (G >= 4) v += dpp<kDppQuadXor2>(v);
  if constexpr (G >= 8) v += dpp<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp<kDppRowMirror>(v);
  return v;
}

// Minimum over aligned groups of G lanes (G in {1,2,4,8,16}); every lane of
// the group receives it.  All lanes of the wave must be active.
template <int G>
__device__ inline uint32_t group_min(uint32_t v) {
  if constexpr (G >= 2) v = min(v, dpp<kDppQuadXor1>(v));
  if constexpr (G >= 4) v = min(v, dpp<kDppQuadXor2>(v));
  if constexpr (G >= 8) v = min(v, dpp<kDppHalfMirror>(v));
  if constexpr (G >= 16) v = min(v, dpp<kDppRowMirror>(v));
  return v;
}

// Exclusive prefix sum within aligned groups of G lanes (G in {1,2,4,8,16}),
// lane r of a group receiving the sum of lanes 0 .. r-1 (row shifts within
// rows of 16 lanes; a lane adds a shifted value only from its own group).
// All lanes of the wave must be active.
template <int G>
__device__ inline uint32_t group_excl_scan(uint32_t v) {
  const int r = int(__lane_id()) & (G - 1);
  uint32_t incl = v;
  if constexpr (G >= 2) { const uint32_t u = uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x111, 0xF, 0xF, true)); if (r >= 1) incl += u; }
  if constexpr (G >= 4) { const uint32_t u = uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x112, 0xF, 0xF, true)); if (r >= 2) incl += u; }
  if constexpr (G >= 8) { const uint32_t u = uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x114, 0xF, 0xF, true)); if (r >= 4) incl += u; }
  if constexpr (G >= 16) { const uint32_t u = uint32_t(__builtin_amdgcn_update_dpp(0, int(incl), 0x118, 0xF, 0xF, true)); if (r >= 8) incl += u; }
  return incl - v;
}

// Broadcast lane (group base + S) within aligned groups of G lanes (G <= 16).
template <int G, int S>
__device__ inline uint32_t group_bcast(uint32_t v) {
  constexpr int and_mask = 0x1F & ~(G - 1);
  constexpr int pattern = and_mask | (S << 5);
  return uint32_t(__builtin_amdgcn_ds_swizzle(int(v), pattern));
}

}  // namespace blsh
