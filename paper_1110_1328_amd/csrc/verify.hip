// Verification kernels for gfx950: Algorithm 1 (BayesLSH), Algorithm 2
// (BayesLSH-Lite) and the exhaustive comparator.
//
// Every kernel walks the per-candidate loop of the algorithms: compare k
// hashes, add the agreements to m, then look up the decision for (m, n) in the
// precomputed table (minMatches and the concentration cache of Section 4.3).
//
//   k_verify_bits     sign-random-projection signatures (cosine); one lane per
//                     candidate, 4 candidates per lane; level j reads k/32 words
//                     per side (k = 16 reads half a word).  With the word-major
//                     layout the words of one level form a dense slab (4 bytes
//                     per object), so the gathers stay in L2.  With a prefix
//                     view the first 128 hashes come in one 16-byte gather per
//                     side; in Algorithm 1 the candidates left after them go to
//                     a survivor queue for k_verify_tail.
//   k_verify_tail     Algorithm 1 past the prefix, one lane per queued pair.
//   k_verify_minhash  minhash signatures (Jaccard); a group of k/4 lanes compares
//                     one candidate's k hashes with one 16-byte load per lane and
//                     per side, then sums the agreements with DPP; lane l owns
//                     candidate l of the wave's tile of 64.
//   k_exact_*         exact similarity on Lite survivors (one wave per pair).
//   k_exhaustive_*    the comparator: all n_max hashes of both object-major rows,
//                     per-level counts, prefix sums, then the decision sequence
//                     of Algorithm 1/2 replayed (or the classical m/n estimate).
//   k_acc_flush       the accepted pairs staged in slices during a launch,
//                     appended to the caller's list.
//
// Survivor queues and the accepted-pair staging are split into slices whose
// counters sit on separate cache lines (device-common helpers): one counter
// for a whole launch would serialise every wave's atomic.
#include <map>
#include <mutex>

#include "device_common.h"

namespace blsh {

// ---------------------------------------------------------------------------
// SRP: one lane per candidate
// ---------------------------------------------------------------------------
template <int K, bool WORD_MAJOR>
__device__ inline uint32_t level_agree_bits(const VerifyArgs &a, uint32_t xi, uint32_t yi, int j) {
  if constexpr (K == 32) {
    const uint32_t wx = WORD_MAJOR ? a.sig[size_t(j) * a.n_obj + xi] : a.sig[size_t(xi) * a.row_words + j];
    const uint32_t wy = WORD_MAJOR ? a.sig[size_t(j) * a.n_obj + yi] : a.sig[size_t(yi) * a.row_words + j];
    return 32u - __popc(wx ^ wy);
  } else if constexpr (K == 64) {
    const int w0 = 2 * j, w1 = 2 * j + 1;
    uint32_t x0, x1, y0, y1;
    if (WORD_MAJOR) {
      x0 = a.sig[size_t(w0) * a.n_obj + xi];
      x1 = a.sig[size_t(w1) * a.n_obj + xi];
      y0 = a.sig[size_t(w0) * a.n_obj + yi];
      y1 = a.sig[size_t(w1) * a.n_obj + yi];
    } else {
      x0 = a.sig[size_t(xi) * a.row_words + w0];
      x1 = a.sig[size_t(xi) * a.row_words + w1];
      y0 = a.sig[size_t(yi) * a.row_words + w0];
      y1 = a.sig[size_t(yi) * a.row_words + w1];
    }
    return 64u - __popc(x0 ^ y0) - __popc(x1 ^ y1);
  } else {  // K == 16
    const int w = j >> 1;
    const uint32_t wx = WORD_MAJOR ? a.sig[size_t(w) * a.n_obj + xi] : a.sig[size_t(xi) * a.row_words + w];
    const uint32_t wy = WORD_MAJOR ? a.sig[size_t(w) * a.n_obj + yi] : a.sig[size_t(yi) * a.row_words + w];
    const uint32_t d = ((wx ^ wy) >> ((j & 1) * 16)) & 0xFFFFu;
    return 16u - __popc(d);
  }
}

constexpr int kPPT = 4;        // candidates per lane (bits kernel)
constexpr int kBlock = 256;

// agreement of level j from the XOR of the two 16-byte prefixes (in registers)
template <int K>
__device__ inline uint32_t agree_from_xor(const uint32_t *d, int j) {
  if constexpr (K == 32) return 32u - __popc(d[j]);
  else if constexpr (K == 64) return 64u - __popc(d[2 * j]) - __popc(d[2 * j + 1]);
  else return 16u - __popc((d[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu);
}

constexpr int kExactLds = 512;   // entries of the longer sparse row staged in LDS per wave

// Exact similarity of one pair computed by the whole wave (Algorithm 2's
// final step): cosine of dense rows or of sparse rows with sorted indices
// (FP64 sums), or Jaccard of sorted sets (integer counts, one FP64 division).
// Sparse: the longer row is staged in this wave's LDS rows when it fits and
// every entry of the shorter row is binary-searched in it.
__device__ double exact_wave(const VerifyArgs &a, uint32_t xi, uint32_t yi, uint32_t *s_idx, float *s_val) {
  const int lane = lane_id();
  if (a.ex_kind == BLSH_DENSE) {
    const float *u = a.ex_dense + size_t(xi) * a.ex_dim, *v = a.ex_dense + size_t(yi) * a.ex_dim;
    double nx = 0, ny = 0, dot = 0;
    for (int64_t d = lane; d < a.ex_dim; d += kWave) {
      const double p = u[d], q = v[d];
      nx += p * p; ny += q * q; dot += p * q;
    }
    nx = wave_sum_f64(nx); ny = wave_sum_f64(ny); dot = wave_sum_f64(dot);
    return (nx > 0 && ny > 0) ? dot / (sqrt(nx) * sqrt(ny)) : 0.0;
  }
  const int64_t ax = a.ex_offsets[xi], nxl = a.ex_offsets[xi + 1] - ax;
  const int64_t ay = a.ex_offsets[yi], nyl = a.ex_offsets[yi + 1] - ay;
  const bool x_long = nxl >= nyl;
  const int64_t al = x_long ? ax : ay, nl = x_long ? nxl : nyl;
  const int64_t as = x_long ? ay : ax, ns = x_long ? nyl : nxl;
  const bool csr = a.ex_kind == BLSH_CSR;
  const bool staged = nl <= kExactLds;
  double n_long = 0.0, n_short = 0.0, dot = 0.0;
  uint32_t inter = 0;
  if (staged) {
    for (int64_t i = lane; i < nl; i += kWave) {
      s_idx[i] = a.ex_indices[al + i];
      if (csr) {
        const float v = a.ex_values[al + i];
        s_val[i] = v;
        n_long += double(v) * double(v);
      }
    }
    wave_lds_sync();
  } else if (csr) {
    for (int64_t i = lane; i < nl; i += kWave) { const double v = a.ex_values[al + i]; n_long += v * v; }
  }
  for (int64_t i = lane; i < ns; i += kWave) {
    const uint32_t key = a.ex_indices[as + i];
    int64_t lo = 0, hi = nl;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      const uint32_t v = staged ? s_idx[mid] : a.ex_indices[al + mid];
      if (v < key) lo = mid + 1; else hi = mid;
    }
    const bool hit = lo < nl && (staged ? s_idx[lo] : a.ex_indices[al + lo]) == key;
    if (csr) {
      const double vs = a.ex_values[as + i];
      n_short += vs * vs;
      if (hit) dot += vs * double(staged ? s_val[lo] : a.ex_values[al + lo]);
    } else {
      inter += hit;
    }
  }
  wave_lds_sync();   // the wave may stage another row next
  if (csr) {
    n_long = wave_sum_f64(n_long); n_short = wave_sum_f64(n_short); dot = wave_sum_f64(dot);
    const double nx = x_long ? n_long : n_short, ny = x_long ? n_short : n_long;
    return (nx > 0 && ny > 0) ? dot / (sqrt(nx) * sqrt(ny)) : 0.0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) inter += __shfl_xor(inter, o);
  const int64_t uni = nxl + nyl - int64_t(inter);
  return uni > 0 ? double(inter) / double(uni) : 0.0;
}

// Emission of one Lite survivor's exact similarity (called by lane 0): into
// the wave's staging slice, or the caller's list when that is full.
__device__ inline void emit_exact(const VerifyArgs &a, int64_t c, double s) {
  if (!(s > a.t)) return;
  const int sl = wave_slice();
  const unsigned long long spos = atomicAdd((unsigned long long *)(a.acc_cnt + sl * kCntStride), 1ull);
  if (int64_t(spos) < a.st_cap) {
    a.st_rel[size_t(sl) * a.st_cap + spos] = uint32_t(c - a.c_begin);
    a.st_val[size_t(sl) * a.st_cap + spos] = float(s);
    return;
  }
  const unsigned long long pos = atomicAdd((unsigned long long *)a.acc_total, 1ull);
  if (int64_t(pos) < a.acc_cap) {
    a.acc_idx[pos] = uint64_t(c);
    a.acc_val[pos] = float(s);
  } else {
    raise_status(a.status, BLSH_ETRUNCATED);
  }
}

// One lane per candidate, kPPT consecutive candidates per lane.
//   PFX: the first 128 hashes of each side are loaded with one 16-byte gather
//        (from the caller's prefix array or the start of object-major rows), so
//        the first 128/K levels need no further round trip; later levels read
//        `sig` in its own layout.
//   LITE: survivors of the h-hash budget get their exact similarity right here,
//        one survivor at a time by the whole wave (Algorithm 2), or, with
//        TAIL, from k_exact after this kernel.
// (8 waves per SIMD: the register bound costs a few bytes of spill in the
// rarely taken exact-similarity path and keeps more gathers in flight)
// The accept bits of the first kLdsAccLevels levels are staged in LDS (a
// global table load per level and candidate would double the kernel's memory
// instructions); later levels read the table.
constexpr int kLdsAccLevels = 8;
constexpr int kMaxAccWords = (64 * kMaxLevels + 1 + 31) / 32;

// Queue entries of the tail: m | next level << 16, or, with kDecidedBit, m |
// level << 16 of a candidate already accepted inside the prefix (the tail only
// emits it).
constexpr uint32_t kDecidedBit = 1u << 31;

//   TAIL (PFX): a second kernel finishes the work (this kernel then carries
//        no emission code: fewer registers, no spills).  Not LITE: only the
//        prefix levels run here; every candidate still undecided after them,
//        and every one accepted inside them, goes to the survivor queue, and
//        k_verify_tail finishes and emits them.  LITE: the survivors of the h
//        hashes go to the exact-similarity queue for k_exact.
template <int K, int KIND, bool LITE, bool WORD_MAJOR, bool PFX, bool TAIL = false>
__global__ __launch_bounds__(kBlock, 8) void k_verify_bits(VerifyArgs a) {
  static_assert(!TAIL || PFX, "the split follows the prefix");
  constexpr bool FUSED = LITE && !TAIL;   // Lite exact similarity in this kernel
  constexpr int PL = PFX ? 128 / K : 0;   // levels served by the prefix
  __shared__ int s_min[kMaxLevels];
  __shared__ uint32_t s_acc[LITE ? 1 : kLdsAccLevels * kMaxAccWords];
  __shared__ uint32_t s_eidx[FUSED ? kBlock / kWave : 1][FUSED ? kExactLds : 1];
  __shared__ float s_eval[FUSED ? kBlock / kWave : 1][FUSED ? kExactLds : 1];
  const int L = a.n_levels;
  const int words = int(a.table[2]);
  if (threadIdx.x < kMaxLevels)
    s_min[threadIdx.x] = threadIdx.x < L ? int(a.table[kTabMinOff + threadIdx.x]) : 0x7fffffff;
  if constexpr (!LITE) {
    for (int i = threadIdx.x; i < min(L, kLdsAccLevels) * words; i += kBlock) s_acc[i] = a.table[kTabAccOff + i];
  }
  __syncthreads();
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t c0 = a.c_begin + (tile * kBlock + threadIdx.x) * kPPT;
  const bool any = c0 < a.c_end;

  uint32_t xi[kPPT], yi[kPPT];
  uint32_t alive = 0, bad = 0;
#pragma unroll
  for (int p = 0; p < kPPT; ++p) xi[p] = yi[p] = 0;
  if (any) {
    if (KIND == BLSH_PAIRS && c0 + kPPT <= a.c_end && ((uintptr_t(a.x + c0) | uintptr_t(a.y + c0)) & 15) == 0) {
      const u32x4 vx = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.x + c0));
      const u32x4 vy = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.y + c0));
      xi[0] = vx.x; xi[1] = vx.y; xi[2] = vx.z; xi[3] = vx.w;
      yi[0] = vy.x; yi[1] = vy.y; yi[2] = vy.z; yi[3] = vy.w;
#pragma unroll
      for (int p = 0; p < kPPT; ++p) {
        if (xi[p] < a.n_obj && yi[p] < a.n_obj) alive |= 1u << p; else bad |= 1u << p;
      }
    } else {
#pragma unroll
      for (int p = 0; p < kPPT; ++p) {
        if (c0 + p < a.c_end) {
          if (fetch_candidate(a, c0 + p, xi[p], yi[p])) alive |= 1u << p; else bad |= 1u << p;
        }
      }
    }
  }
  uint32_t m[kPPT] = {0, 0, 0, 0};
  uint8_t code[kPPT] = {0, 0, 0, 0};
  uint32_t emit = 0;
  auto decide = [&](int p, int j) {
    if (int(m[p]) < s_min[j]) {
      code[p] = uint8_t((BLSH_PRUNED << 6) | j);
      alive &= ~(1u << p);
    } else if (!LITE && (j < kLdsAccLevels ? (s_acc[j * words + (m[p] >> 5)] >> (m[p] & 31)) & 1u
                                            : accept_bit(a.table, words, j, int(m[p])))) {
      code[p] = uint8_t((BLSH_ACCEPT_CONC << 6) | j);
      alive &= ~(1u << p);
      emit |= 1u << p;
    } else if (j == L - 1) {
      code[p] = uint8_t(((LITE ? BLSH_LITE_EXACT : BLSH_ACCEPT_NMAX) << 6) | j);
      alive &= ~(1u << p);
      emit |= 1u << p;
    }
  };
  int j0 = 0;
  if constexpr (PFX) {
    // all eight gathers are issued before any is consumed (object 0 stands in
    // for candidates that are out of range or invalid; their result is unused)
    // (address: one 32 x 32 -> 64-bit multiply-add per gather).  A lane's
    // consecutive candidates usually share x (bucket-major rows, query
    // lists): its x prefix is then reused rather than gathered again, and a
    // wave in which no lane needs it skips the load.
    u32x4 hx[kPPT], hy[kPPT];
    const char *pb = reinterpret_cast<const char *>(a.pfx);
    const uint32_t sb = uint32_t(a.pfx_stride) * 4u;
    uint32_t ex[kPPT];
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
      const uint32_t ok = 0u - ((alive >> p) & 1u);
      ex[p] = xi[p] & ok;
      hy[p] = *reinterpret_cast<const u32x4 *>(pb + uint64_t(yi[p] & ok) * sb);
    }
    hx[0] = *reinterpret_cast<const u32x4 *>(pb + uint64_t(ex[0]) * sb);
#pragma unroll
    for (int p = 1; p < kPPT; ++p) {
      hx[p] = hx[p - 1];
      if (ex[p] != ex[p - 1]) hx[p] = *reinterpret_cast<const u32x4 *>(pb + uint64_t(ex[p]) * sb);
    }
    uint32_t d[kPPT][4];
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
      d[p][0] = hx[p].x ^ hy[p].x; d[p][1] = hx[p].y ^ hy[p].y;
      d[p][2] = hx[p].z ^ hy[p].z; d[p][3] = hx[p].w ^ hy[p].w;
    }
    for (int j = 0; j < PL && j < L && alive; ++j) {
#pragma unroll
      for (int p = 0; p < kPPT; ++p) {
        if (!(alive & (1u << p))) continue;
        m[p] += agree_from_xor<K>(d[p], j);
        decide(p, j);
      }
    }
    j0 = PL;
    if constexpr (TAIL && !LITE) {
      // still undecided after the prefix, or accepted inside it: to the
      // queue, finished by k_verify_tail with every lane busy (the code
      // written below is overwritten there)
      uint32_t mj[kPPT];
#pragma unroll
      for (int p = 0; p < kPPT; ++p)
        mj[p] = (alive >> p) & 1u ? m[p] | (uint32_t(j0) << 16)
                                  : m[p] | (uint32_t(code[p] & 63) << 16) | kDecidedBit;
      push_survivors<kPPT>(a, alive | emit, c0, mj);
      alive = 0;
      emit = 0;
    }
  }
  for (int j = j0; j < L && alive; ++j) {
#pragma unroll
    for (int p = 0; p < kPPT; ++p)
      if (alive & (1u << p)) m[p] += level_agree_bits<K, WORD_MAJOR>(a, xi[p], yi[p], j);
#pragma unroll
    for (int p = 0; p < kPPT; ++p)
      if (alive & (1u << p)) decide(p, j);
  }
#pragma unroll
  for (int p = 0; p < kPPT; ++p)
    if (bad & (1u << p)) code[p] = 0xFF;
  if (bad) raise_status(a.status, BLSH_EBADID);

  if (any) {
    if (c0 + kPPT <= a.c_end && (uintptr_t(a.code + c0) & 3) == 0) {
      const uint32_t packed = uint32_t(code[0]) | (uint32_t(code[1]) << 8) | (uint32_t(code[2]) << 16) |
                              (uint32_t(code[3]) << 24);
      __builtin_nontemporal_store(packed, reinterpret_cast<uint32_t *>(a.code + c0));
    } else {
#pragma unroll
      for (int p = 0; p < kPPT; ++p)
        if (c0 + p < a.c_end) a.code[c0 + p] = code[p];
    }
    if (a.m_dbg) {
#pragma unroll
      for (int p = 0; p < kPPT; ++p)
        if (c0 + p < a.c_end) a.m_dbg[c0 + p] = uint16_t(m[p]);
    }
  }
  if constexpr (TAIL) {
    if constexpr (LITE) {
#pragma unroll
      for (int p = 0; p < kPPT; ++p) push_survivor(a, (emit >> p) & 1u, c0 + p);
    }
    return;
  }
  // emission in converged control flow
  if (__ballot(emit != 0) == 0) return;
  if constexpr (LITE) {
    // the survivors' ids are fetched again (wave-uniform, rare) rather than
    // kept in registers through the exact-similarity code
    const int w = threadIdx.x / kWave;
    const int64_t wave_c0 = a.c_begin + (tile * kBlock + int64_t(w) * kWave) * kPPT;
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
      uint64_t mask = __ballot((emit >> p) & 1u);
      while (mask) {
        const int l = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int64_t c = wave_c0 + int64_t(l) * kPPT + p;
        uint32_t sx, sy;
        if constexpr (KIND == BLSH_PAIRS) {
          sx = a.x[c];
          sy = a.y[c];
        } else {
          fetch_candidate(a, c, sx, sy);
        }
        const double sim = exact_wave(a, sx, sy, s_eidx[w], s_eval[w]);
        if (lane_id() == 0) emit_exact(a, c, sim);
      }
    }
  } else {
    const double alpha = tab_f64(a.table, 4), beta = tab_f64(a.table, 6);
#pragma unroll
    for (int p = 0; p < kPPT; ++p) {
      const bool e = (emit >> p) & 1u;
      const int n = ((code[p] & 63) + 1) * K;
      const float v = e ? map_estimate(a.measure, int(m[p]), n, alpha, beta) : 0.f;
      emit_accepted(a, e, uint64_t(c0 + p), v);
    }
  }
}

// ---------------------------------------------------------------------------
// Minhash: a group of K/4 lanes per candidate
// ---------------------------------------------------------------------------
template <int G, int S>
struct MinhashStep {
  template <int K>
  __device__ static inline void run(const VerifyArgs &a, uint32_t xi, uint32_t yi, uint32_t alive, int j, int r,
                                    uint32_t &own) {
    const uint32_t xs = group_bcast<G, S>(xi);
    const uint32_t ys = group_bcast<G, S>(yi);
    const uint32_t al = group_bcast<G, S>(alive);
    uint32_t c = 0;
    if (al) {
      const uint4 hx = *reinterpret_cast<const uint4 *>(a.sig + size_t(xs) * a.row_words + j * K + 4 * r);
      const uint4 hy = *reinterpret_cast<const uint4 *>(a.sig + size_t(ys) * a.row_words + j * K + 4 * r);
      c = uint32_t(hx.x == hy.x) + uint32_t(hx.y == hy.y) + uint32_t(hx.z == hy.z) + uint32_t(hx.w == hy.w);
    }
    c = group_sum<G>(c);
    if (r == S) own = c;
    if constexpr (S + 1 < G) MinhashStep<G, S + 1>::template run<K>(a, xi, yi, alive, j, r, own);
  }
};

template <int K, int KIND, bool LITE>
__global__ __launch_bounds__(kBlock) void k_verify_minhash(VerifyArgs a) {
  constexpr int G = K / 4;
  __shared__ int s_min[kMaxLevels];
  if (threadIdx.x < kMaxLevels)
    s_min[threadIdx.x] = threadIdx.x < a.n_levels ? int(a.table[kTabMinOff + threadIdx.x]) : 0x7fffffff;
  __syncthreads();
  const int L = a.n_levels;
  const int words = int(a.table[2]);
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t c = a.c_begin + tile * kBlock + threadIdx.x;
  const int lane = lane_id();
  const int r = lane & (G - 1);
  if (__ballot(c < a.c_end) == 0) return;  // whole wave past the end

  uint32_t xi = 0, yi = 0, alive = 0;
  bool bad = false;
  if (c < a.c_end) {
    if (fetch_candidate(a, c, xi, yi)) alive = 1; else { bad = true; xi = yi = 0; }
  }
  uint32_t m = 0;
  uint8_t code = bad ? 0xFF : 0;
  bool emit = false;
  for (int j = 0; j < L; ++j) {
    if (__ballot(alive != 0) == 0) break;
    uint32_t own = 0;
    MinhashStep<G, 0>::template run<K>(a, xi, yi, alive, j, r, own);
    if (alive) {
      m += own;
      if (int(m) < s_min[j]) {
        code = uint8_t((BLSH_PRUNED << 6) | j);
        alive = 0;
      } else if (!LITE && accept_bit(a.table, words, j, int(m))) {
        code = uint8_t((BLSH_ACCEPT_CONC << 6) | j);
        alive = 0;
        emit = true;
      } else if (j == L - 1) {
        code = uint8_t(((LITE ? BLSH_LITE_EXACT : BLSH_ACCEPT_NMAX) << 6) | j);
        alive = 0;
        emit = true;
      }
    }
  }
  if (bad) raise_status(a.status, BLSH_EBADID);
  if (c < a.c_end) {
    a.code[c] = code;
    if (a.m_dbg) a.m_dbg[c] = uint16_t(m);
  }
  if (LITE) {
    push_survivor(a, emit, c);
  } else {
    const double alpha = tab_f64(a.table, 4), beta = tab_f64(a.table, 6);
    const float v = emit ? map_estimate(a.measure, int(m), ((code & 63) + 1) * K, alpha, beta) : 0.f;
    emit_accepted(a, emit, uint64_t(c), v);
  }
}

// ---------------------------------------------------------------------------
// Exact similarity on Lite survivors: one wave per queued pair
// ---------------------------------------------------------------------------



// One wave per queued pair (Lite survivors of the minhash and exhaustive paths).
// The grid holds a multiple of kSlices waves: wave g serves queue slice
// g % kSlices together with the other waves of that slice.
__global__ __launch_bounds__(kBlock) void k_exact(VerifyArgs a) {
  __shared__ uint32_t s_idx[kBlock / kWave][kExactLds];
  __shared__ float s_val[kBlock / kWave][kExactLds];
  const int w = threadIdx.x >> 6;
  const int64_t g = int64_t(blockIdx.x) * (kBlock / kWave) + w;
  const int sl = int(g % kSlices);
  const int64_t parts = int64_t(gridDim.x) * (kBlock / kWave) / kSlices;
  const int64_t n = min(a.q_cnt[sl * kCntStride], a.q_cap);
  const uint32_t *rel = a.q_rel + size_t(sl) * a.q_cap;
  for (int64_t q = g / kSlices; q < n; q += parts) {
    const int64_t c = a.c_begin + rel[q];
    uint32_t xi, yi;
    fetch_candidate(a, c, xi, yi);   // ids were range-checked before the pair was queued
    const double sim = exact_wave(a, xi, yi, s_idx[w], s_val[w]);
    if (lane_id() == 0) emit_exact(a, c, sim);
  }
}

// Algorithm 1 for the SRP candidates queued after the 128-hash prefix: one
// lane per queued pair, from its next level on.  Layouts (LM):
//   kTailWM     word-major slabs, where every word is a gather of its own: a
//               step loads one level's words;
//   kTailRow16  object-major rows of a multiple of 4 words, 16-byte aligned: a
//               step loads the next two 16-byte chunks of both sides, every
//               load issued before any is used, so one round trip serves
//               256 / K levels;
//   kTailRow4   other object-major rows (a caller's prefix array beside rows
//               that a 16-byte load cannot start, e.g. 160 or 192 hashes): the
//               same 8-word step read one word at a time, never past the row.
// minMatches and the accept bits sit in LDS (the decision of a level costs no
// memory round trip).
// Agreeing hashes of level q of the 8 loaded words (q < 256 / K; q is a
// constant after unrolling, so every word index is too).
template <int K>
__device__ inline uint32_t agree_at(const uint32_t (&d)[8], int q) {
  if constexpr (K == 32) return 32u - __popc(d[q]);
  else if constexpr (K == 64) return 64u - __popc(d[2 * q]) - __popc(d[2 * q + 1]);
  else return 16u - __popc((d[q >> 1] >> ((q & 1) * 16)) & 0xFFFFu);
}

constexpr int kTailWM = 0, kTailRow16 = 1, kTailRow4 = 2;

template <int K, int LM>
__global__ __launch_bounds__(kBlock) void k_verify_tail(VerifyArgs a) {
  constexpr bool WM = LM == kTailWM;
  extern __shared__ uint32_t s_acc[];   // n_levels * words accept-bit words
  __shared__ int s_min[kMaxLevels];
  const int L = a.n_levels;
  const int words = int(a.table[2]);
  if (threadIdx.x < kMaxLevels)
    s_min[threadIdx.x] = threadIdx.x < L ? int(a.table[kTabMinOff + threadIdx.x]) : 0x7fffffff;
  for (int i = threadIdx.x; i < L * words; i += kBlock) s_acc[i] = a.table[kTabAccOff + i];
  __syncthreads();
  const double alpha = tab_f64(a.table, 4), beta = tab_f64(a.table, 6);
  constexpr int kStepWords = WM ? (K == 64 ? 2 : 1) : 8;   // words of each side per step
  constexpr int kStepLevels = kStepWords * 32 / K;
  // the grid is a multiple of kSlices blocks: block b serves queue slice
  // b % kSlices together with the other blocks of that slice
  const int sl = int(blockIdx.x % kSlices);
  const int64_t n = min(a.q_cnt[sl * kCntStride], a.q_cap);
  const uint32_t *rel = a.q_rel + size_t(sl) * a.q_cap;
  const uint32_t *qm = a.q_m + size_t(sl) * a.q_cap;
  const int64_t stride = int64_t(gridDim.x / kSlices) * kBlock;
  for (int64_t i0 = int64_t(blockIdx.x / kSlices) * kBlock; i0 < n; i0 += stride) {
    const int64_t i = i0 + threadIdx.x;
    int64_t c = 0;
    uint32_t m = 0;
    uint8_t code = 0;
    bool emit = false;
    if (i < n) {
      c = a.c_begin + rel[i];
      const uint32_t e = qm[i];
      m = e & 0xFFFFu;
      int j = int((e >> 16) & 0x7FFFu);
      bool done = false;
      uint32_t x = 0, y = 0;
      if (e & kDecidedBit) {   // accepted inside the prefix: emit only
        code = uint8_t((BLSH_ACCEPT_CONC << 6) | j);
        emit = done = true;
      } else if (a.kind == BLSH_PAIRS) {
        x = a.x[c];
        y = a.y[c];
      } else {
        fetch_candidate(a, c, x, y);
      }
      while (!done) {
        // words [w0, w0 + 8) of both sides (w0: first word of level j; a
        // 16-byte chunk boundary for rows)
        int w0 = j * K / 32;
        if constexpr (!WM) w0 &= ~3;
        const int base = w0 * 32 / K;   // level of the first loaded hashes
        const int avail = min(kStepWords, a.row_words - w0);
        uint32_t d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (WM) {
          uint32_t hx[kStepWords], hy[kStepWords];
#pragma unroll
          for (int u = 0; u < kStepWords; ++u) {
            hx[u] = a.sig[size_t(w0 + u) * a.n_obj + x];
            hy[u] = a.sig[size_t(w0 + u) * a.n_obj + y];
          }
#pragma unroll
          for (int u = 0; u < kStepWords; ++u) d[u] = hx[u] ^ hy[u];
        } else if constexpr (LM == kTailRow4) {
          const uint32_t *rx = a.sig + size_t(x) * a.row_words + w0, *ry = a.sig + size_t(y) * a.row_words + w0;
          uint32_t hx[8], hy[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            hx[u] = u < avail ? rx[u] : 0u;
            hy[u] = u < avail ? ry[u] : 0u;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) d[u] = hx[u] ^ hy[u];
        } else {
          const u32x4 hx0 = *reinterpret_cast<const u32x4 *>(a.sig + size_t(x) * a.row_words + w0);
          const u32x4 hy0 = *reinterpret_cast<const u32x4 *>(a.sig + size_t(y) * a.row_words + w0);
          u32x4 hx1 = hx0, hy1 = hy0;
          if (avail > 4) {
            hx1 = *reinterpret_cast<const u32x4 *>(a.sig + size_t(x) * a.row_words + w0 + 4);
            hy1 = *reinterpret_cast<const u32x4 *>(a.sig + size_t(y) * a.row_words + w0 + 4);
          }
          d[0] = hx0.x ^ hy0.x; d[1] = hx0.y ^ hy0.y; d[2] = hx0.z ^ hy0.z; d[3] = hx0.w ^ hy0.w;
          d[4] = hx1.x ^ hy1.x; d[5] = hx1.y ^ hy1.y; d[6] = hx1.z ^ hy1.z; d[7] = hx1.w ^ hy1.w;
        }
        const int q0 = j - base, qn = min(L - base, avail * 32 / K);
#pragma unroll
        for (int q = 0; q < kStepLevels; ++q) {
          if (q >= q0 && q < qn && !done) {
            m += agree_at<K>(d, q);
            const int jj = base + q;
            if (int(m) < s_min[jj]) {
              code = uint8_t((BLSH_PRUNED << 6) | jj);
              done = true;
            } else if ((s_acc[jj * words + (m >> 5)] >> (m & 31)) & 1u) {
              code = uint8_t((BLSH_ACCEPT_CONC << 6) | jj);
              emit = done = true;
            } else if (jj == L - 1) {
              code = uint8_t((BLSH_ACCEPT_NMAX << 6) | jj);
              emit = done = true;
            }
          }
        }
        j = base + qn;
      }
      a.code[c] = code;
      if (a.m_dbg) a.m_dbg[c] = uint16_t(m);
    }
    const float v = emit ? map_estimate(a.measure, int(m), ((code & 63) + 1) * K, alpha, beta) : 0.f;
    emit_accepted(a, emit, uint64_t(c), v);
  }
}

// Exact similarity of every candidate in [c_begin, c_end), one wave per pair,
// written to out[c] in FP64 (bad ids: NaN and BLSH_EBADID).
__global__ __launch_bounds__(kBlock) void k_exact_pairs(VerifyArgs a, double *out) {
  __shared__ uint32_t s_idx[kBlock / kWave][kExactLds];
  __shared__ float s_val[kBlock / kWave][kExactLds];
  const int w = threadIdx.x >> 6;
  const int64_t waves = int64_t(gridDim.x) * (kBlock / kWave);
  for (int64_t c = a.c_begin + int64_t(blockIdx.x) * (kBlock / kWave) + w; c < a.c_end; c += waves) {
    uint32_t xi, yi;
    if (!fetch_candidate(a, c, xi, yi)) {
      if (lane_id() == 0) {
        out[c] = __builtin_nan("");
        raise_status(a.status, BLSH_EBADID);
      }
      continue;
    }
    const double sim = exact_wave(a, xi, yi, s_idx[w], s_val[w]);
    if (lane_id() == 0) out[c] = sim;
  }
}

// ---------------------------------------------------------------------------
// Bucket tiles (BLSH_TILES, SRP): a wave takes one 16 x 16 tile of a bucket's
// member pairs at a time.
//   stage   the first n_max hashes (NW words) of the tile's 32 members go to
//           the wave's LDS: 16-byte chunks, consecutive lanes on consecutive
//           chunks of a row, so each 128-byte line is one load -- 32 lines per
//           tile instead of two gathers per pair;
//   level 0 lane l owns positions p = 4l .. 4l+3 (row l/4, columns 4(l%4) ..
//           4(l%4)+3) and decides level 0, and level 1's prune, from the
//           staged first words, writing the codes of the pairs it decides;
//           the positions still open are listed in LDS;
//   rest    groups of P2 lanes take the listed pairs, each lane WPL words of
//           both rows from LDS (128/K levels per 4 words), count agreements
//           per level, prefix them across the group and find the first level
//           that decides (prune below minMatches; accept at or above the
//           minimum accepting m, or by the accept bits when a level's accept
//           set is not an interval; n_max); the group takes the earliest,
//           writes the pair's code and stages it if accepted.
// Waves are persistent; the waves of an XCD sweep contiguous windows of tiles
// together, so a bucket's rows stay in that XCD's L2 while its tiles pass.
// ---------------------------------------------------------------------------
constexpr uint32_t kNoObject = 0xFFFFFFFFu;
constexpr int kTileWords = int(sizeof(blsh_tile) / 4);   // 48: the descriptor, one dword per lane
static_assert(sizeof(blsh_tile) == 192, "tile descriptor layout");

// LDS of one wave: the tile's rows (padded by 4 words so that the groups'
// 16-byte reads of different rows spread over the banks) and the listed pairs
// (rank << 8 | position).
template <int NW>
struct TileLds {
  uint32_t rows[32][NW + 4];
  uint16_t list[256 + kWave];   // entries 256.. take the stores of lanes with nothing to list
};

// *(T *)((char *)base + off): a 32-bit byte offset from a wave-uniform base
// (one address register per lane instead of a 64-bit sum)
template <class T>
__device__ inline T &at_byte(T *base, uint32_t off) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}

// A field of the kernel's VerifyArgs argument (its first, at offset 0 of
// the kernel-argument segment) read where it is used, not held in scalar
// registers through the kernel: for the fields of rare paths (bad ids, the
// debug array, a full staging region) in a kernel at the scalar register
// limit, whose spilled scalars would otherwise be reloaded on every tile.
template <class T>
__device__ inline T arg_on_use(size_t off) {
  const auto *kp = (const char __attribute__((address_space(4))) *)__builtin_amdgcn_kernarg_segment_ptr();
  return *reinterpret_cast<const volatile T __attribute__((address_space(4))) *>(kp + off);
}
#define BLSH_ARG_ON_USE(f) arg_on_use<decltype(VerifyArgs::f)>(offsetof(VerifyArgs, f))

// LITE (Algorithm 2): the table has no accept sets, so a listed pair is
// pruned at some level or reaches the last one (n = h); those get the Lite
// code and go to the wave's staging region with their ids, for k_tiles_exact.
// The host sizes a Lite launch so that no region can fill.
// Occupancy: a wave waits for its staging loads on every tile, and resident
// waves cover those waits; interval tables at K >= 32 and up to 1024 bits
// are held to 72 registers, seven waves per SIMD (measured best; eight would
// not fit the LDS, 4 waves' rows and lists per block).
template <int K, int NW, bool INTERVALS, bool LITE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(INTERVALS && K >= 32 && NW <= 32 ? 7 : 1))) void k_verify_tiles(VerifyArgs a) {
  constexpr int P2 = NW >= 16 ? NW / 8 : 1;   // lanes per listed pair
  constexpr int WPL = NW / P2;                // words per lane (4 or 8)
  constexpr int LPL = WPL * 32 / K;           // levels per lane
  constexpr int SPI = kWave / P2;             // listed pairs per wave step
  constexpr int CPO = NW / 4;                 // 16-byte chunks per staged row
  constexpr int NCH = 32 * CPO;               // chunks per tile
  constexpr int CPL = (NCH + kWave - 1) / kWave;
  static_assert(kWave % CPO == 0, "a lane's chunks sit at one offset within their rows");
  __shared__ TileLds<NW> lds_all[kBlock / kWave];
  TileLds<NW> &S = lds_all[threadIdx.x >> 6];
  extern __shared__ uint32_t s_acc[];         // accept bits (tables with non-interval accept sets)
  const int L = a.n_levels;
  const int words = int(a.table[2]);
  if (!INTERVALS)
    for (int i = threadIdx.x; i < L * words; i += kBlock) s_acc[i] = a.table[kTabAccOff + i];
  __syncthreads();
  const int lane = lane_id(), q = lane % P2, g = lane / P2;
  // level j's tests in disagreements D (hashes that differ among the first
  // (j+1) K, so m = (j+1) K - D): prune iff D > pd[j], accept iff D <= ad[j]
  // (pd = (j+1) K - minMatches, ad = (j+1) K - min_accept; either may be -1:
  // always prune / never accept); in LDS, read 4 levels at a time.  With
  // interval accept sets a level continues iff ad < D <= pd, one unsigned
  // test of D - lo against w (lo = ad + 1, w = pd - ad), also in LDS.
  __shared__ int4 s_pd[kMaxLevels / 4], s_ad[kMaxLevels / 4];
  __shared__ uint4 s_lo[kMaxLevels / 4], s_w[kMaxLevels / 4];
  if (threadIdx.x < kMaxLevels) {
    const int j = threadIdx.x, n = (j + 1) * K;
    const int pd = j < L ? n - int(a.table[kTabMinOff + j]) : -1, ad = j < L ? n - int(a.table[kTabAloOff + j]) : -1;
    reinterpret_cast<int *>(s_pd)[j] = pd;
    reinterpret_cast<int *>(s_ad)[j] = ad;
    reinterpret_cast<uint32_t *>(s_lo)[j] = uint32_t(ad + 1);
    reinterpret_cast<uint32_t *>(s_w)[j] = uint32_t(pd - ad);
  }
  __syncthreads();
  const bool last_lane = q == P2 - 1;         // holds level L - 1 as its level LPL - 1
  const uint32_t min0 = a.table[kTabMinOff];
  // level 1's prune test in the first pass (none with a single level), after
  // level 0's accept test: ad0 = K - min_accept of level 0
  const uint32_t min1 = L > 1 ? a.table[kTabMinOff + 1] : 0u;
  const int ad0 = reinterpret_cast<const int *>(s_ad)[0];
  const int gw = int(xcd_tile(blockIdx.x, gridDim.x)) * (kBlock / kWave) +
                 __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kWave);
  const int n_waves = int(gridDim.x) * (kBlock / kWave);
  // the launch's tiles (at most 2^22, numbered from t_begin) as a buffer of
  // 192-byte descriptors: 32-bit offsets, one dword per lane
  const int n_t = int(a.t_end - a.t_begin);
  const __amdgpu_buffer_rsrc_t tile_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<blsh_tile *>(a.tiles + a.t_begin), 0, n_t * int(sizeof(blsh_tile)), 0x00020000);
  // the signature rows as a buffer (gfx9 raw buffer, 32-bit data format word);
  // offsets past its size read zeros
  const __amdgpu_buffer_rsrc_t sig_rsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(a.sig), 0, int(a.sig_buf_bytes), 0x00020000);
  const int r = lane >> 2, cc = 16 + 4 * (lane & 3);   // level 0: row r, staged rows cc .. cc+3
  // this wave's staging region: accepted pairs (candidate index, raw
  // m | n << 16) in order; past its end, the caller's list directly
  // (a region holds fewer than 2^29 entries: 32-bit counts and byte offsets)
  uint64_t *w_idx = a.st_idx + size_t(gw) * a.st_cap;
  float *w_val = a.st_val + size_t(gw) * a.st_cap;
  uint2 *w_xy = LITE ? a.st_xy + size_t(gw) * a.st_cap : nullptr;
  const uint32_t st_cap = uint32_t(a.st_cap);
  uint32_t w_cnt = 0;   // wave-uniform
  // the descriptor, one dword per lane, loaded one tile ahead
  uint32_t nd = 0;
  if (gw < n_t && lane < kTileWords)
    nd = __builtin_amdgcn_raw_buffer_load_b32(tile_rsrc, 4 * lane, uint32_t(gw) * uint32_t(sizeof(blsh_tile)), 0);
  for (int t = gw; t < n_t; t += n_waves) {   // wave-uniform
    const uint32_t dw = nd;
    if (t + n_waves < n_t && lane < kTileWords)
      nd = __builtin_amdgcn_raw_buffer_load_b32(tile_rsrc, 4 * lane, uint32_t(t + n_waves) * uint32_t(sizeof(blsh_tile)),
                                                0);
    const int64_t first = int64_t(uint64_t(uint32_t(__builtin_amdgcn_readlane(int(dw), 0))) |
                                  (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(dw), 1))) << 32));
    const int n_rows = __builtin_amdgcn_readlane(int(dw), 2), n_cols = __builtin_amdgcn_readlane(int(dw), 3);
    // member ids (lanes 0..31) and this lane's four keep bits (positions 4l .. 4l+3)
    const uint32_t idv = uint32_t(__shfl(int(dw), 12 + (lane & 31)));
    const uint32_t kb = (uint32_t(__shfl(int(dw), 4 + (lane >> 3))) >> (4 * (lane & 7))) & 0xFu;
    const bool member = lane < 32 && (lane & 15) < (lane < 16 ? n_rows : n_cols);
    const uint32_t id = member && idv < a.n_obj ? idv : kNoObject;
    if (member && idv >= a.n_obj) raise_status(BLSH_ARG_ON_USE(status), BLSH_EBADID);
    // stage the rows (a missing member stages object 0's row, never read):
    // every chunk's load is issued before the first is stored
    // (chunk lane + 64 u is chunk lane % CPO of row lane / CPO + u 64 / CPO:
    // one address register per lane, the rest immediate offsets)
    const uint32_t idz = id == kNoObject ? 0u : id;
    uint32_t oid[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u)   // lanes past the last chunk read a lane they do not use
      oid[u] = uint32_t(__builtin_amdgcn_ds_bpermute(4 * (lane / CPO) + 4 * u * (kWave / CPO), int(idz)));
    u32x4 chunk[CPL];
    if (a.sig_buf_bytes) {   // wave-uniform: one 24-bit multiply-add per chunk
      const uint32_t row_bytes = uint32_t(a.row_words) * 4u, lane_off = 16u * uint32_t(lane % CPO);
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (NCH % kWave == 0 || lane + kWave * u < NCH) {
          const auto v = __builtin_amdgcn_raw_buffer_load_b128(sig_rsrc, __umul24(oid[u], row_bytes) + lane_off, 0, 0);
          chunk[u] = u32x4{v[0], v[1], v[2], v[3]};
        }
    } else {
      const uint32_t *sig_l = a.sig + 4 * (lane % CPO);
#pragma unroll
      for (int u = 0; u < CPL; ++u)
        if (NCH % kWave == 0 || lane + kWave * u < NCH)
          chunk[u] = *reinterpret_cast<const u32x4 *>(sig_l + uint64_t(oid[u]) * uint32_t(a.row_words));
    }
#pragma unroll
    for (int u = 0; u < CPL; ++u)
      if (NCH % kWave == 0 || lane + kWave * u < NCH)
        *reinterpret_cast<u32x4 *>(&S.rows[lane / CPO + u * (kWave / CPO)][4 * (lane % CPO)]) = chunk[u];
    const uint32_t xid = uint32_t(__builtin_amdgcn_ds_bpermute(4 * r, int(id)));
    uint32_t yid[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) yid[i] = uint32_t(__builtin_amdgcn_ds_bpermute(4 * cc + 4 * i, int(id)));
    // ranks: kept positions in lower lanes (all slots), then this lane's lower slots
    int below = 0, count = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t b = __ballot((kb >> i) & 1u);
      below += int(lanes_below(b));
      count += __popcll(b);
    }
    wave_lds_sync();
    if (first < 0 || first + count > a.n_cand) {   // numbering outside the call's candidates: the tile is skipped
      if (lane == 0) raise_status(BLSH_ARG_ON_USE(status), BLSH_EINVAL);
      continue;
    }
    // levels 0 and 1 for this lane's four positions (2K <= 128 hashes: the
    // first 4 words of each row, one LDS read): a pair pruned at level 0, or
    // at level 1 without level 0 having accepted it, is decided here and its
    // code written; the rest is listed and written once decided.  The tile's
    // candidates are the run [first, first + count), by rank.
    uint8_t *const cb = a.code + first;
    const u32x4 xw = *reinterpret_cast<const u32x4 *>(&S.rows[r][0]);
    uint32_t surv = 0, mm[4];
    bool malformed = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rk = below + __popc(kb & ((1u << i) - 1u));
      const bool kept = (kb >> i) & 1u;
      const bool ok = xid != kNoObject && yid[i] != kNoObject;
      const u32x4 yw = *reinterpret_cast<const u32x4 *>(&S.rows[cc + i][0]);
      uint32_t m0, m1;
      if constexpr (K == 16) {
        const uint32_t d = xw.x ^ yw.x;
        m0 = 16u - __popc(d & 0xFFFFu);
        m1 = 16u - __popc(d >> 16);
      } else if constexpr (K == 32) {
        m0 = 32u - __popc(xw.x ^ yw.x);
        m1 = 32u - __popc(xw.y ^ yw.y);
      } else {
        m0 = 64u - __popc(xw.x ^ yw.x) - __popc(xw.y ^ yw.y);
        m1 = 64u - __popc(xw.z ^ yw.z) - __popc(xw.w ^ yw.w);
      }
      const bool s0 = kept && ok && m0 >= min0;
      const bool acc0 = INTERVALS ? int(K - m0) <= ad0 : ((s_acc[m0 >> 5] >> (m0 & 31)) & 1u) != 0;
      const bool p1 = s0 && !acc0 && m0 + m1 < min1;
      mm[i] = p1 ? m0 + m1 : m0;
      if (kept && !(s0 && !p1))
        at_byte(cb, uint32_t(rk)) = ok ? uint8_t((BLSH_PRUNED << 6) | (p1 ? 1 : 0)) : uint8_t(0xFF);
      malformed |= kept && !ok && (r >= n_rows || cc - 16 + i >= n_cols);   // a position past the tile's members
      surv |= uint32_t(s0 && !p1) << i;
    }
    if (malformed) raise_status(BLSH_ARG_ON_USE(status), BLSH_EINVAL);
    if (uint16_t *const m_dbg = BLSH_ARG_ON_USE(m_dbg)) {   // m of the pairs level 0 decides (survivors: after their last level)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if ((kb >> i) & 1u) m_dbg[first + below + __popc(kb & ((1u << i) - 1u))] = uint16_t(mm[i]);
    }
    // the surviving positions (rank << 8 | position), in position order
    int at = 0, total = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint64_t b = __ballot((surv >> i) & 1u);
      at += int(lanes_below(b));
      total += __popcll(b);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool sv = (surv >> i) & 1u;
      S.list[sv ? at : 256 + lane] = uint16_t(((below + __popc(kb & ((1u << i) - 1u))) << 8) | (4 * lane + i));
      at += int(sv);
    }
    wave_lds_sync();
    // the listed pairs over their whole rows
    for (int base = 0; base < total; base += SPI) {   // wave-uniform
      const int e = base + g;
      const bool act = e < total;
      const uint32_t ent = act ? S.list[e] : 0u;
      const int p = int(ent & 0xFFu), rk = int(ent >> 8);
      const uint32_t *xr = &S.rows[p >> 4][q * WPL];
      const uint32_t *yr = &S.rows[16 + (p & 15)][q * WPL];
      uint32_t d[WPL];
#pragma unroll
      for (int w4 = 0; w4 < WPL; w4 += 4) {
        const u32x4 hx = *reinterpret_cast<const u32x4 *>(xr + w4);
        const u32x4 hy = *reinterpret_cast<const u32x4 *>(yr + w4);
        d[w4] = hx.x ^ hy.x; d[w4 + 1] = hx.y ^ hy.y; d[w4 + 2] = hx.z ^ hy.z; d[w4 + 3] = hx.w ^ hy.w;
      }
      // disagreements cumulated over this lane's levels, then over the group's
      // lower lanes
      int D[LPL];
      uint32_t acc = 0;
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        if constexpr (K == 16) acc += __popc((d[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu);
        else if constexpr (K == 32) acc += __popc(d[i]);
        else acc += __popc(d[2 * i]) + __popc(d[2 * i + 1]);
        D[i] = int(acc);
      }
      const int pre = int(group_excl_scan<P2>(acc));
      // the first deciding level of this lane (scanned from the last, so the
      // earliest wins): key = level << 20 | D; the decision itself is read
      // off (j, D) afterwards.
      uint32_t key = 0xFFFFFFFFu;
      if constexpr (INTERVALS) {
        // this lane's bounds, read on every step rather than held in registers
        // through the tile (the opaque index keeps the reads in the loop):
        // fewer live registers, more resident waves
        int bi = q * LPL / 4;
        asm volatile("" : "+v"(bi));
        uint32_t lo[LPL], w[LPL];
#pragma unroll
        for (int i4 = 0; i4 < LPL; i4 += 4) {
          const uint4 vl = s_lo[bi + i4 / 4], vw = s_w[bi + i4 / 4];
          lo[i4] = vl.x; lo[i4 + 1] = vl.y; lo[i4 + 2] = vl.z; lo[i4 + 3] = vl.w;
          w[i4] = vw.x; w[i4 + 1] = vw.y; w[i4 + 2] = vw.z; w[i4 + 3] = vw.w;
        }
        const uint32_t kb0 = uint32_t(q * LPL) << 20;
#pragma unroll
        for (int i = LPL - 1; i >= 0; --i) {
          const uint32_t Di = uint32_t(D[i] + pre);
          const bool decide = Di - lo[i] >= w[i] || (i == LPL - 1 && last_lane);
          key = decide ? kb0 + (uint32_t(i) << 20) + Di : key;
        }
      } else {
#pragma unroll
        for (int i = LPL - 1; i >= 0; --i) {
          const int Di = D[i] + pre;
          const int j = q * LPL + i;
          const int m = (j + 1) * K - Di;
          const bool prune = Di > reinterpret_cast<const int *>(s_pd)[j];
          const bool accept = !prune && ((s_acc[j * words + (m >> 5)] >> (m & 31)) & 1u);
          key = (prune || accept || (i == LPL - 1 && last_lane)) ? ((uint32_t(j) << 20) | uint32_t(Di)) : key;
        }
      }
      key = group_min<P2>(key);
      const int j = int(key >> 20), Dj = int(key & 0xFFFFFu), m = (j + 1) * K - Dj;
      int dec;
      if (Dj > reinterpret_cast<const int *>(s_pd)[j]) dec = BLSH_PRUNED;
      else if (INTERVALS ? Dj <= reinterpret_cast<const int *>(s_ad)[j] : ((s_acc[j * words + (m >> 5)] >> (m & 31)) & 1u))
        dec = BLSH_ACCEPT_CONC;
      else dec = LITE ? BLSH_LITE_EXACT : BLSH_ACCEPT_NMAX;
      const bool lead = act && q == 0;
      if (lead) {
        at_byte(cb, uint32_t(rk)) = uint8_t((dec << 6) | j);
        if (uint16_t *const m_dbg = BLSH_ARG_ON_USE(m_dbg)) m_dbg[first + rk] = uint16_t(m);
      }
      const bool emit = lead && dec != BLSH_PRUNED;
      const uint64_t em = __ballot(emit);
      const uint32_t pos = w_cnt + lanes_below(em);
      if constexpr (LITE) {
        // the pair's ids for its exact similarity (every lane takes part in the shuffles)
        const uint32_t ix = uint32_t(__shfl(int(id), p >> 4)), iy = uint32_t(__shfl(int(id), 16 + (p & 15)));
        if (emit && pos < st_cap) {   // (the host sizes the launch so that it always is)
          at_byte(w_idx, pos * 8u) = uint64_t(first + rk);
          at_byte(w_xy, pos * 8u) = make_uint2(ix, iy);
        } else if (emit) {
          raise_status(BLSH_ARG_ON_USE(status), BLSH_EINVAL);
        }
      } else {
        // S_hat is computed from (m, n) when the staging is flushed
        const bool over = emit && pos >= st_cap;
        if (emit && !over) {
          at_byte(w_idx, pos * 8u) = uint64_t(first + rk);
          at_byte(w_val, pos * 4u) = __uint_as_float(uint32_t(m) | (uint32_t((j + 1) * K) << 16));
        }
        if (__ballot(over)) {   // the region is full: S_hat here, into the caller's list
          VerifyArgs r{};   // the fields emit_direct reads, read here
          r.acc_idx = BLSH_ARG_ON_USE(acc_idx);
          r.acc_val = BLSH_ARG_ON_USE(acc_val);
          r.acc_cap = BLSH_ARG_ON_USE(acc_cap);
          r.acc_total = BLSH_ARG_ON_USE(acc_total);
          r.status = BLSH_ARG_ON_USE(status);
          const uint32_t *tab = BLSH_ARG_ON_USE(table);
          const float sv = over ? map_estimate(BLSH_ARG_ON_USE(measure), m, (j + 1) * K, tab_f64(tab, 4), tab_f64(tab, 6)) : 0.f;
          emit_direct(r, over, uint64_t(first + rk), sv);
        }
      }
      w_cnt += uint32_t(__popcll(em));
    }
    wave_lds_sync();   // the next tile's staging overwrites these rows and lists
  }
  if (lane == 0) a.wst_cnt[gw] = min(w_cnt, st_cap);
}

// Tiles path, after each launch: the waves' staging counts, exclusive prefix
// from the running accepted count (which already holds the pairs that went to
// the caller's list directly); the running count advances past them, and on
// the call's last launch becomes *n_acc.  One block.
__global__ __launch_bounds__(1024) void k_tiles_scan(const uint32_t *cnt, int64_t n_waves, int64_t *off,
                                                      int64_t *total, int64_t *n_acc, int last) {
  __shared__ int64_t s_part[1024 / kWave];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) s_carry = *total;
  __syncthreads();
  for (int64_t b0 = 0; b0 < n_waves; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < n_waves ? int64_t(cnt[i]) : 0;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t u = __shfl_up(x, o);
      if (lane_id() >= o) x += u;
    }
    if (lane_id() == kWave - 1) s_part[threadIdx.x / kWave] = x;
    __syncthreads();
    int64_t before = s_carry;
    for (int w = 0; w < int(threadIdx.x / kWave); ++w) before += s_part[w];
    if (i < n_waves) off[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *total = s_carry;
    if (last) *n_acc = s_carry;
  }
}

// Tiles path, Lite: the exact similarity of every pair a wave of the tile
// kernel staged (Algorithm 2's final step); those with s > t are compacted to
// the front of the region with s as their value, and the region's count
// becomes theirs.  One block per region, its waves taking the pairs in rounds
// of one pair each: every entry of a round is read before any is written, and
// a round writes only slots below its own entries, so the compaction never
// overwrites an entry not yet read.
__global__ __launch_bounds__(kBlock) void k_tiles_exact(VerifyArgs a) {
  __shared__ uint32_t s_idx[kBlock / kWave][kExactLds];
  __shared__ float s_val[kBlock / kWave][kExactLds];
  __shared__ int s_kept;
  const int64_t w = blockIdx.x;
  const int wv = threadIdx.x >> 6;
  const int64_t n = a.wst_cnt[w];
  uint64_t *idx = a.st_idx + size_t(w) * a.st_cap;
  float *val = a.st_val + size_t(w) * a.st_cap;
  const uint2 *xy = a.st_xy + size_t(w) * a.st_cap;
  if (threadIdx.x == 0) s_kept = 0;
  __syncthreads();
  for (int64_t r0 = 0; r0 < n; r0 += kBlock / kWave) {   // uniform over the block
    const int64_t e = r0 + wv;
    const bool has = e < n;
    uint64_t c = 0;
    uint2 p = make_uint2(0, 0);
    if (has) {
      c = idx[e];
      p = xy[e];
    }
    __syncthreads();
    if (has) {
      const double sim = exact_wave(a, p.x, p.y, s_idx[wv], s_val[wv]);
      if (lane_id() == 0 && sim > a.t) {
        const int slot = atomicAdd(&s_kept, 1);
        idx[slot] = c;
        val[slot] = float(sim);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) a.wst_cnt[w] = uint32_t(s_kept);
}

// Tiles path: each wave's staged accepted pairs to the caller's list at its
// offset, S_hat computed from (m, n) (Lite: the exact similarity staged);
// one block per wave region.
__global__ __launch_bounds__(kBlock) void k_tiles_copy(VerifyArgs a, const int64_t *off) {
  const int64_t w = blockIdx.x;
  const int64_t n = a.wst_cnt[w], base = off[w];
  const double alpha = tab_f64(a.table, 4), beta = tab_f64(a.table, 6);
  const uint64_t *idx = a.st_idx + size_t(w) * a.st_cap;
  const float *val = a.st_val + size_t(w) * a.st_cap;
  bool trunc = false;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    const int64_t pos = base + i;
    if (pos < a.acc_cap) {
      const uint32_t u = __float_as_uint(val[i]);
      a.acc_idx[pos] = idx[i];
      a.acc_val[pos] = a.st_raw ? map_estimate(a.measure, int(u & 0xFFFFu), int(u >> 16), alpha, beta) : val[i];
    } else {
      trunc = true;
    }
  }
  if (trunc) raise_status(a.status, BLSH_ETRUNCATED);
}

// ---------------------------------------------------------------------------
// Exhaustive comparator
// ---------------------------------------------------------------------------
// Decision replay over cumulative counts: returns true when level j with m
// agreements ends the per-candidate loop, and sets the decision.
__device__ inline bool replay_decides(const VerifyArgs &a, const int *s_min, int words, int j, int m, int &dec) {
  const int L = a.n_levels;
  if (m < s_min[j]) { dec = BLSH_PRUNED; return true; }
  if (a.mode == BLSH_REPLAY) {
    if (accept_bit(a.table, words, j, m)) { dec = BLSH_ACCEPT_CONC; return true; }
    if (j == L - 1) { dec = BLSH_ACCEPT_NMAX; return true; }
  } else if (j == L - 1) {
    dec = BLSH_LITE_EXACT;
    return true;
  }
  return false;
}

// SRP rows of W words (W % 4 == 0, W <= 64): G = W/4 lanes per candidate, one
// 16-byte load per lane and side; lane r holds words 4r..4r+3.
template <int K, int G>
__global__ __launch_bounds__(kBlock) void k_exhaustive_bits(VerifyArgs a) {
  __shared__ int s_min[kMaxLevels];
  if (threadIdx.x < kMaxLevels)
    s_min[threadIdx.x] = threadIdx.x < a.n_levels ? int(a.table[kTabMinOff + threadIdx.x]) : 0x7fffffff;
  __syncthreads();
  constexpr int PPW = kWave / G;            // candidates per wave step
  constexpr int LPL = 128 / K;              // levels per lane
  const int words = int(a.table[2]);
  const int lane = lane_id(), r = lane % G, g = lane / G;
  const int64_t wave = (xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / kWave;
  const int64_t c = a.c_begin + wave * PPW + g;
  const bool in = c < a.c_end;
  uint32_t xi = 0, yi = 0;
  bool ok = false;
  if (in) ok = fetch_candidate(a, c, xi, yi);
  // per-level agreement counts of this lane's 128 bits
  uint32_t cnt[LPL];
  uint32_t tot = 0;
  if (ok && 4 * r < a.row_words) {
    const uint4 hx = *reinterpret_cast<const uint4 *>(a.sig + size_t(xi) * a.row_words + 4 * r);
    const uint4 hy = *reinterpret_cast<const uint4 *>(a.sig + size_t(yi) * a.row_words + 4 * r);
    const uint32_t d[4] = {hx.x ^ hy.x, hx.y ^ hy.y, hx.z ^ hy.z, hx.w ^ hy.w};
#pragma unroll
    for (int q = 0; q < LPL; ++q) {
      if constexpr (K == 16) cnt[q] = 16u - __popc((d[q >> 1] >> ((q & 1) * 16)) & 0xFFFFu);
      else if constexpr (K == 32) cnt[q] = 32u - __popc(d[q]);
      else cnt[q] = 64u - __popc(d[2 * q]) - __popc(d[2 * q + 1]);
      tot += cnt[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < LPL; ++q) cnt[q] = 0;
  }
  // exclusive prefix of lane totals within the group
  uint32_t incl = tot;
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o, G);
    if (r >= o) incl += v;
  }
  uint32_t run = incl - tot;
  const int L = a.n_levels;
  int dec = -1, dj = 0, dm = 0;
  if (a.mode == BLSH_MLE) {
    uint32_t total = __shfl(incl, g * G + G - 1);
    dm = int(total);
    dj = a.count_levels - 1;
    dec = -2;  // resolved below by lane r == 0
  } else {
#pragma unroll
    for (int q = 0; q < LPL; ++q) {
      run += cnt[q];
      const int j = r * LPL + q;
      int d;
      if (dec < 0 && j < L && replay_decides(a, s_min, words, j, int(run), d)) { dec = d; dj = j; dm = int(run); }
    }
  }
  // first deciding lane of the group
  const uint64_t has = __ballot(dec >= 0);
  const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (g * G);
  const uint64_t mine = has & gmask;
  const int first = mine ? __ffsll((unsigned long long)mine) - 1 : g * G;
  const int fdec = __shfl(dec, first), fj = __shfl(dj, first), fm = __shfl(dm, first);
  bool emit = false, surv = false;
  float val = 0.f;
  if (in && r == 0) {
    uint8_t code;
    if (!ok) {
      code = 0xFF;
      raise_status(a.status, BLSH_EBADID);
    } else if (a.mode == BLSH_MLE) {
      const int n = a.count_levels * K;
      double s = double(fm) / n;
      if (a.measure == BLSH_COSINE) s = cos(3.14159265358979323846 * (1.0 - s));
      emit = s >= a.t;
      val = float(s);
      code = uint8_t(((emit ? BLSH_ACCEPT_NMAX : BLSH_PRUNED) << 6) | fj);
    } else {
      code = uint8_t((fdec << 6) | fj);
      if (fdec == BLSH_ACCEPT_CONC || fdec == BLSH_ACCEPT_NMAX) {
        emit = true;
        val = map_estimate(a.measure, fm, (fj + 1) * K, tab_f64(a.table, 4), tab_f64(a.table, 6));
      } else if (fdec == BLSH_LITE_EXACT) {
        surv = true;
      }
    }
    a.code[c] = code;
    if (a.m_dbg) a.m_dbg[c] = uint16_t(fm);
  }
  if (a.mode == BLSH_REPLAY_LITE) push_survivor(a, surv, c);
  else emit_accepted(a, emit, uint64_t(c), val);
}

// Minhash rows of H <= 256 hashes: one candidate per wave step, lane r holds
// hashes 4r..4r+3; a wave-wide prefix gives the cumulative count at each level.
template <int K>
__global__ __launch_bounds__(kBlock) void k_exhaustive_minhash(VerifyArgs a) {
  __shared__ int s_min[kMaxLevels];
  if (threadIdx.x < kMaxLevels)
    s_min[threadIdx.x] = threadIdx.x < a.n_levels ? int(a.table[kTabMinOff + threadIdx.x]) : 0x7fffffff;
  __syncthreads();
  constexpr int LPG = K / 4;                 // lanes per level
  const int words = int(a.table[2]);
  const int lane = lane_id();
  const int64_t wave = (xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / kWave;
  const int64_t c = a.c_begin + wave;
  if (c >= a.c_end) return;                  // wave-uniform
  uint32_t xi = 0, yi = 0;
  const bool ok = fetch_candidate(a, c, xi, yi);
  uint32_t cnt = 0;
  const int H = a.count_levels * K;
  if (ok && 4 * lane < H) {
    const uint4 hx = *reinterpret_cast<const uint4 *>(a.sig + size_t(xi) * a.row_words + 4 * lane);
    const uint4 hy = *reinterpret_cast<const uint4 *>(a.sig + size_t(yi) * a.row_words + 4 * lane);
    cnt = uint32_t(hx.x == hy.x) + uint32_t(hx.y == hy.y) + uint32_t(hx.z == hy.z) + uint32_t(hx.w == hy.w);
  }
  uint32_t incl = cnt;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t v = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += v;
  }
  const int L = a.n_levels;
  int dec = -1, dj = 0, dm = 0;
  const int j = lane / LPG;
  if (a.mode != BLSH_MLE && (lane % LPG) == LPG - 1 && j < L) {
    int d;
    if (replay_decides(a, s_min, words, j, int(incl), d)) { dec = d; dj = j; dm = int(incl); }
  }
  const uint64_t has = __ballot(dec >= 0);
  const int first = has ? __ffsll((unsigned long long)has) - 1 : 0;
  const int fdec = __shfl(dec, first), fj = __shfl(dj, first), fm = __shfl(dm, first);
  const uint32_t total = __shfl(incl, kWave - 1);
  bool emit = false, surv = false;
  float val = 0.f;
  if (lane == 0) {
    uint8_t code;
    int mval = fm;
    if (!ok) {
      code = 0xFF;
      raise_status(a.status, BLSH_EBADID);
    } else if (a.mode == BLSH_MLE) {
      const double s = double(total) / H;
      emit = s >= a.t;
      val = float(s);
      mval = int(total);
      code = uint8_t(((emit ? BLSH_ACCEPT_NMAX : BLSH_PRUNED) << 6) | (a.count_levels - 1));
    } else {
      code = uint8_t((fdec << 6) | fj);
      if (fdec == BLSH_ACCEPT_CONC || fdec == BLSH_ACCEPT_NMAX) {
        emit = true;
        val = map_estimate(a.measure, fm, (fj + 1) * K, tab_f64(a.table, 4), tab_f64(a.table, 6));
      } else if (fdec == BLSH_LITE_EXACT) {
        surv = true;
      }
    }
    a.code[c] = code;
    if (a.m_dbg) a.m_dbg[c] = uint16_t(mval);
  }
  if (a.mode == BLSH_REPLAY_LITE) push_survivor(a, surv, c);
  else emit_accepted(a, emit, uint64_t(c), val);
}

__global__ void k_zero_i64(int64_t *p) {
  if (threadIdx.x == 0) *p = 0;
}

// Clears every counter of the single-call paths (both staging-count sets and
// running counts, the queue counts): one block of kSlices threads.  Only
// needed after a call that stopped before its last flush.
__global__ void k_zero_slices(int64_t *cnt) {
  for (int i = 0; i < 3; ++i) cnt[(size_t(i) * kSlices + threadIdx.x) * kCntStride] = 0;
  if (threadIdx.x < 2) cnt[(size_t(3) * kSlices + threadIdx.x) * kCntStride] = 0;
}

// After each launch (chunk), one block per staging slice, no atomics: every
// block reads the kSlices counts of the launch's staging set (a.acc_cnt) and
// the running count (*a.acc_total), and block s copies slice s to the
// caller's list after the slices before it.  The next launch uses the other
// set (nxt_cnt, *nxt_total): block 0 clears its counts and stores the new
// running count there, or 0 and *n_acc on the call's last launch.  Block s
// also clears queue count s.
// kFlushParts blocks share a slice, each copying a contiguous part of it.
constexpr int kFlushParts = 8;

__global__ __launch_bounds__(kBlock) void k_acc_flush(VerifyArgs a, int64_t *nxt_cnt, int64_t *nxt_total, int last) {
  static_assert(kSlices == kBlock, "one staging slice per thread of a block");
  __shared__ int64_t s_cnt[kSlices];
  __shared__ int64_t s_base, s_total;
  const int t = threadIdx.x, sl = blockIdx.x % kSlices, part = blockIdx.x / kSlices;
  int64_t c = min(a.acc_cnt[size_t(t) * kCntStride], a.st_cap);
  // inclusive scan of the slice counts across the block (wave scan, then
  // the four wave totals)
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
  s_cnt[t] = before + v - c;   // exclusive prefix
  if (t == kSlices - 1) s_total = before + v;
  if (t == 0) s_base = *a.acc_total;
  __syncthreads();
  const int64_t n = min(a.acc_cnt[size_t(sl) * kCntStride], a.st_cap);
  const int64_t base = s_base + s_cnt[sl];
  const uint32_t *rel = a.st_rel + size_t(sl) * a.st_cap;
  const float *val = a.st_val + size_t(sl) * a.st_cap;
  const int64_t cb = a.c_begin;
  const double alpha = tab_f64(a.table, 4), beta = tab_f64(a.table, 6);
  const int64_t per = (n + kFlushParts - 1) / kFlushParts;
  const int64_t i1 = min(n, (part + 1) * per);
  bool trunc = false;
  for (int64_t i = part * per + t; i < i1; i += kBlock) {
    const int64_t pos = base + i;
    if (pos < a.acc_cap) {
      a.acc_idx[pos] = uint64_t(cb) + rel[i];
      float v = val[i];
      if (a.st_raw) {   // S_hat from (m, n), one pair per lane
        const uint32_t u = __float_as_uint(v);
        v = map_estimate(a.measure, int(u & 0xFFFFu), int(u >> 16), alpha, beta);
      }
      a.acc_val[pos] = v;
    } else {
      trunc = true;
    }
  }
  if (trunc) raise_status(a.status, BLSH_ETRUNCATED);
  if (part == 0 && t == 0 && a.q_cnt) a.q_cnt[size_t(sl) * kCntStride] = 0;
  if (sl == 0 && part == 0) {
    nxt_cnt[size_t(t) * kCntStride] = 0;
    if (t == 0) {
      const int64_t total = s_base + s_total;
      *nxt_total = last ? 0 : total;
      if (last) *a.n_acc = total;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int64_t blocks_for(int64_t items, int64_t per_block) { return (items + per_block - 1) / per_block; }

template <int K, bool LITE, bool WM, bool PFX, bool TAIL = false>
static int launch_bits_kind(const VerifyArgs &a, int64_t nb, hipStream_t s) {
  switch (a.kind) {
    case BLSH_PAIRS: hipLaunchKernelGGL((k_verify_bits<K, BLSH_PAIRS, LITE, WM, PFX, TAIL>), dim3(nb), dim3(kBlock), 0, s, a); break;
    case BLSH_QUERY_LISTS: hipLaunchKernelGGL((k_verify_bits<K, BLSH_QUERY_LISTS, LITE, WM, PFX, TAIL>), dim3(nb), dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL((k_verify_bits<K, BLSH_ALL_PAIRS, LITE, WM, PFX, TAIL>), dim3(nb), dim3(kBlock), 0, s, a); break;
  }
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

// tail: the prefix kernel hands the rest of the work to a second kernel
// through the survivor queue (Algorithm 1: a.q_m set, k_verify_tail; Lite:
// a.q_rel set, k_exact)
template <int K, bool LITE>
static int launch_bits_layout(const VerifyArgs &a, int64_t nb, bool wm, bool pfx, bool tail, hipStream_t s) {
  if (tail) return wm ? launch_bits_kind<K, LITE, true, true, true>(a, nb, s)
                      : launch_bits_kind<K, LITE, false, true, true>(a, nb, s);
  if (wm) return pfx ? launch_bits_kind<K, LITE, true, true>(a, nb, s) : launch_bits_kind<K, LITE, true, false>(a, nb, s);
  return pfx ? launch_bits_kind<K, LITE, false, true>(a, nb, s) : launch_bits_kind<K, LITE, false, false>(a, nb, s);
}

template <int K, bool LITE>
static int launch_minhash_kind(const VerifyArgs &a, int64_t nb, hipStream_t s) {
  switch (a.kind) {
    case BLSH_PAIRS: hipLaunchKernelGGL((k_verify_minhash<K, BLSH_PAIRS, LITE>), dim3(nb), dim3(kBlock), 0, s, a); break;
    case BLSH_QUERY_LISTS: hipLaunchKernelGGL((k_verify_minhash<K, BLSH_QUERY_LISTS, LITE>), dim3(nb), dim3(kBlock), 0, s, a); break;
    default: hipLaunchKernelGGL((k_verify_minhash<K, BLSH_ALL_PAIRS, LITE>), dim3(nb), dim3(kBlock), 0, s, a); break;
  }
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

int launch_verify(blsh_ctx *ctx, const VerifyArgs &a, int k, bool lite, bool word_major, hipStream_t s) {
  const int64_t n = a.c_end - a.c_begin;
  if (n <= 0) return BLSH_OK;
  if (a.measure == BLSH_COSINE) {
    const int64_t nb = blocks_for(n, int64_t(kBlock) * kPPT);
    // the first 128 hashes in one 16-byte gather per side where a prefix view exists
    const bool pfx = a.pfx != nullptr;
    const bool tail = pfx && (lite ? a.q_rel != nullptr : a.q_m != nullptr);
    LaunchScope ls(ctx, s, pfx ? "verify_bits_prefix" : "verify_bits");
#define BLSH_B(KK, LL) if (k == KK && lite == LL) return launch_bits_layout<KK, LL>(a, nb, word_major, pfx, tail, s);
    BLSH_B(16, false) BLSH_B(16, true) BLSH_B(32, false) BLSH_B(32, true) BLSH_B(64, false) BLSH_B(64, true)
#undef BLSH_B
  } else {
    const int64_t nb = blocks_for(n, kBlock);
    LaunchScope ls(ctx, s, "verify_minhash");
#define BLSH_M(KK, LL) if (k == KK && lite == LL) return launch_minhash_kind<KK, LL>(a, nb, s);
    BLSH_M(16, false) BLSH_M(16, true) BLSH_M(32, false) BLSH_M(32, true) BLSH_M(64, false) BLSH_M(64, true)
#undef BLSH_M
  }
  return fail(BLSH_EINVAL, "unsupported k=%d", k);
}

int launch_exhaustive(blsh_ctx *ctx, const VerifyArgs &a, int k, hipStream_t s) {
  const int64_t n = a.c_end - a.c_begin;
  if (n <= 0) return BLSH_OK;
  if (a.measure == BLSH_COSINE) {
    const int G = (a.count_levels * k / 32) / 4;  // lanes per candidate: n_max bits, 128 per lane
    LaunchScope ls(ctx, s, "exhaustive_bits");
    const int64_t nb = blocks_for(n, int64_t(kBlock / G));
#define BLSH_E(KK, GG) if (k == KK && G == GG) { hipLaunchKernelGGL((k_exhaustive_bits<KK, GG>), dim3(nb), dim3(kBlock), 0, s, a); return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE; }
    BLSH_E(16, 1) BLSH_E(16, 2) BLSH_E(16, 4) BLSH_E(16, 8) BLSH_E(16, 16)
    BLSH_E(32, 1) BLSH_E(32, 2) BLSH_E(32, 4) BLSH_E(32, 8) BLSH_E(32, 16)
    BLSH_E(64, 1) BLSH_E(64, 2) BLSH_E(64, 4) BLSH_E(64, 8) BLSH_E(64, 16)
#undef BLSH_E
    return fail(BLSH_EINVAL, "exhaustive: unsupported signature width %d words", a.row_words);
  }
  LaunchScope ls(ctx, s, "exhaustive_minhash");
  const int64_t nb = blocks_for(n, kBlock / kWave);
  if (k == 16) hipLaunchKernelGGL((k_exhaustive_minhash<16>), dim3(nb), dim3(kBlock), 0, s, a);
  else if (k == 32) hipLaunchKernelGGL((k_exhaustive_minhash<32>), dim3(nb), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_exhaustive_minhash<64>), dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

// Grids of the queue consumers: a multiple of kSlices waves (k_exact) or
// blocks (k_verify_tail), at least one per slice.
static inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int launch_exact(blsh_ctx *ctx, const VerifyArgs &a, int64_t max_items, hipStream_t s) {
  if (max_items <= 0) return BLSH_OK;
  const int64_t nb = round_up(std::min<int64_t>(blocks_for(max_items, kBlock / kWave), int64_t(ctx->n_cu) * 16),
                              kSlices / (kBlock / kWave));
  LaunchScope ls(ctx, s, "exact");
  hipLaunchKernelGGL(k_exact, dim3(nb), dim3(kBlock), 0, s, a);
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

// words: accept-bit words per level of the launch's table (LDS of the tail).
// Object-major rows take 16-byte chunk loads only when every row starts on a
// 16-byte boundary and holds a whole number of chunks.
int launch_verify_tail(blsh_ctx *ctx, const VerifyArgs &a, int k, bool word_major, int words, hipStream_t s) {
  const int64_t nb = round_up(int64_t(ctx->n_cu) * 16, kSlices);
  const size_t lds = size_t(a.n_levels) * words * 4;
  const bool row16 = a.row_words % 4 == 0 && (uintptr_t(a.sig) & 15) == 0;
  LaunchScope ls(ctx, s, "verify_tail");
#define BLSH_T(KK)                                                                                          \
  if (k == KK) {                                                                                            \
    if (word_major) hipLaunchKernelGGL((k_verify_tail<KK, kTailWM>), dim3(nb), dim3(kBlock), lds, s, a);     \
    else if (row16) hipLaunchKernelGGL((k_verify_tail<KK, kTailRow16>), dim3(nb), dim3(kBlock), lds, s, a);  \
    else hipLaunchKernelGGL((k_verify_tail<KK, kTailRow4>), dim3(nb), dim3(kBlock), lds, s, a);             \
    return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;                                        \
  }
  BLSH_T(16) BLSH_T(32) BLSH_T(64)
#undef BLSH_T
  return fail(BLSH_EINVAL, "unsupported k=%d", k);
}

// Tiles: the persistent tile kernel over tiles [a.t_begin, a.t_end); NW =
// n_max / 32 words staged per member; accept bits in LDS only for tables whose
// accept sets are not intervals.
// The persistent grid of a tile-kernel variant: as many blocks as stay
// resident on the device at once (occupancy queried once per variant).
template <typename F>
static int64_t resident_blocks(blsh_ctx *ctx, F kernel, size_t lds) {
  static std::mutex mu;
  static std::map<std::pair<const void *, size_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  const auto key = std::make_pair(reinterpret_cast<const void *>(kernel), lds);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, lds) != hipSuccess || per_cu < 1)
      per_cu = 1;
    it = cache.emplace(key, per_cu).first;
  }
  return int64_t(it->second) * ctx->n_cu;
}

// Waves of the persistent tile grid for (k, n_max) (the staging holds one
// region per wave).
int tiles_grid_waves(blsh_ctx *ctx, int k, int n_max, bool intervals, bool lite, size_t lds, int64_t *waves) {
  const int NW = n_max / 32;
#define BLSH_TG(KK, WW)                                                                                        \
  if (k == KK && NW == WW) {                                                                                   \
    *waves = (lite ? resident_blocks(ctx, k_verify_tiles<KK, WW, true, true>, 0)                               \
              : intervals ? resident_blocks(ctx, k_verify_tiles<KK, WW, true, false>, 0)                       \
                          : resident_blocks(ctx, k_verify_tiles<KK, WW, false, false>, lds)) * (kBlock / kWave); \
    return BLSH_OK;                                                                                            \
  }
  BLSH_TG(16, 4) BLSH_TG(16, 8) BLSH_TG(16, 16) BLSH_TG(16, 32) BLSH_TG(16, 64)
  BLSH_TG(32, 4) BLSH_TG(32, 8) BLSH_TG(32, 16) BLSH_TG(32, 32) BLSH_TG(32, 64)
  BLSH_TG(64, 4) BLSH_TG(64, 8) BLSH_TG(64, 16) BLSH_TG(64, 32) BLSH_TG(64, 64)
#undef BLSH_TG
  return fail(BLSH_EINVAL, "tiles: unsupported k=%d, n_max=%d", k, n_max);
}

// grid_waves: from tiles_grid_waves (every wave of the grid writes its count).
// lite: Algorithm 2 (its table's accept sets are empty, so intervals).
int launch_verify_tiles(blsh_ctx *ctx, const VerifyArgs &a, int k, int n_max, int words, bool intervals, bool lite,
                        int64_t grid_waves, hipStream_t s) {
  const int64_t nb = grid_waves / (kBlock / kWave);
  const size_t lds = intervals || lite ? 0 : size_t(a.n_levels) * words * 4;
  const int NW = n_max / 32;
  LaunchScope ls(ctx, s, "verify_tiles");
#define BLSH_TT(KK, WW)                                                                                      \
  if (k == KK && NW == WW) {                                                                                 \
    if (lite) hipLaunchKernelGGL((k_verify_tiles<KK, WW, true, true>), dim3(nb), dim3(kBlock), 0, s, a);      \
    else if (intervals) hipLaunchKernelGGL((k_verify_tiles<KK, WW, true, false>), dim3(nb), dim3(kBlock), 0, s, a); \
    else hipLaunchKernelGGL((k_verify_tiles<KK, WW, false, false>), dim3(nb), dim3(kBlock), lds, s, a);     \
    return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;                                         \
  }
  BLSH_TT(16, 4) BLSH_TT(16, 8) BLSH_TT(16, 16) BLSH_TT(16, 32) BLSH_TT(16, 64)
  BLSH_TT(32, 4) BLSH_TT(32, 8) BLSH_TT(32, 16) BLSH_TT(32, 32) BLSH_TT(32, 64)
  BLSH_TT(64, 4) BLSH_TT(64, 8) BLSH_TT(64, 16) BLSH_TT(64, 32) BLSH_TT(64, 64)
#undef BLSH_TT
  return fail(BLSH_EINVAL, "tiles: unsupported k=%d, n_max=%d", k, n_max);
}

// Tiles path, Lite: the staged pairs' exact similarities, one block per region.
int launch_tiles_exact(blsh_ctx *ctx, const VerifyArgs &a, int64_t grid_waves, hipStream_t s) {
  LaunchScope ls(ctx, s, "tiles_exact");
  hipLaunchKernelGGL(k_tiles_exact, dim3(grid_waves), dim3(kBlock), 0, s, a);
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

// Tiles path, after each launch: offsets of the waves' staged pairs, then the
// copy to the caller's list.
int launch_tiles_flush(blsh_ctx *ctx, const VerifyArgs &a, int64_t grid_waves, int64_t *off, bool last,
                       hipStream_t s) {
  LaunchScope ls(ctx, s, "tiles_flush");
  hipLaunchKernelGGL(k_tiles_scan, dim3(1), dim3(1024), 0, s, a.wst_cnt, grid_waves, off, a.acc_total, a.n_acc,
                     int(last));
  hipLaunchKernelGGL(k_tiles_copy, dim3(grid_waves), dim3(kBlock), 0, s, a, off);
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

int launch_exact_pairs(blsh_ctx *ctx, const VerifyArgs &a, double *out, hipStream_t s) {
  const int64_t n = a.c_end - a.c_begin;
  if (n <= 0) return BLSH_OK;
  const int64_t nb = std::min<int64_t>(blocks_for(n, kBlock / kWave), int64_t(ctx->n_cu) * 16);
  LaunchScope ls(ctx, s, "exact_pairs");
  hipLaunchKernelGGL(k_exact_pairs, dim3(nb), dim3(kBlock), 0, s, a, out);
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

int launch_zero_slices(blsh_ctx *ctx, int64_t *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_slices, dim3(1), dim3(kSlices), 0, s, cnt);
  (void)ctx;
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

int launch_acc_flush(blsh_ctx *ctx, const VerifyArgs &a, int64_t *nxt_cnt, int64_t *nxt_total, bool last,
                     hipStream_t s) {
  LaunchScope ls(ctx, s, "acc_flush");
  hipLaunchKernelGGL(k_acc_flush, dim3(kSlices * kFlushParts), dim3(kBlock), 0, s, a, nxt_cnt, nxt_total, int(last));
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

int launch_zero(blsh_ctx *ctx, int64_t *p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(64), 0, s, p);
  (void)ctx;
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

}  // namespace blsh
