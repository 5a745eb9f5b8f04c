// SRP verification with a block-persistent LDS cache of signature words.
//
// Candidates that come out of LSH banding are bucket-major: a run of
// consecutive pairs draws both of its objects from one bucket's few hundred
// members.  Each block here owns one contiguous range of 2048-candidate tiles
// and keeps, across its tiles, a direct-mapped LDS table of the first three
// signature words of recently seen objects (slot = {id, w0, w1, w2}).  A
// candidate looks its two objects up in the table; only misses gather from
// global memory, and they refill their slot after the tile.  Reads and writes
// of the table are separated by block barriers, so a lookup never sees a
// half-written slot.  The next tile's candidate ids are loaded while the
// current tile is compared.  Decisions are those of Algorithms 1 and 2.
#include "device_common.h"

namespace blsh {

constexpr int kPcBlock = 512;
constexpr int kPcPPT = 4;
constexpr int kPcTile = kPcBlock * kPcPPT;
constexpr int kPcSlotBits = 12;
constexpr int kPcSlots = 1 << kPcSlotBits;
constexpr int kPcWords = 3;
constexpr uint32_t kPcEmpty = 0xFFFFFFFFu;   // never a valid id

template <bool WM>
__device__ inline uint32_t sig_word(const VerifyArgs &a, uint32_t id, int w) {
  return WM ? a.sig[size_t(w) * a.n_obj + id] : a.sig[size_t(id) * a.row_words + w];
}

// words [w0, w0 + n) of level j
template <int K>
__device__ inline int level_first_word(int j) { return K == 16 ? (j >> 1) : j * (K / 32); }
template <int K>
__device__ inline int level_words(int) { return K == 64 ? 2 : 1; }

template <int K>
__device__ inline uint32_t agree_from(const uint32_t *wx, const uint32_t *wy, int j) {
  const int f = level_first_word<K>(j);
  if constexpr (K == 32) return 32u - __popc(wx[f] ^ wy[f]);
  else if constexpr (K == 64) return 64u - __popc(wx[f] ^ wy[f]) - __popc(wx[f + 1] ^ wy[f + 1]);
  else return 16u - __popc(((wx[f] ^ wy[f]) >> ((j & 1) * 16)) & 0xFFFFu);
}

template <int K, int KIND, bool LITE, bool WM>
__global__ __launch_bounds__(kPcBlock, 4) void k_verify_bits_pc(VerifyArgs a, int64_t n_tiles) {
  __shared__ uint4 s_slot[kPcSlots];
  __shared__ int s_min[kMaxLevels];
  for (int i = threadIdx.x; i < kPcSlots; i += kPcBlock) s_slot[i] = make_uint4(kPcEmpty, 0, 0, 0);
  if (threadIdx.x < kMaxLevels)
    s_min[threadIdx.x] = threadIdx.x < a.n_levels ? int(a.table[kTabMinOff + threadIdx.x]) : 0x7fffffff;
  __syncthreads();
  const int L = a.n_levels;
  const int words = int(a.table[2]);
  const int cw = min(kPcWords, a.row_words);        // words cached per object
  const double alpha = tab_f64(a.table, 4), beta = tab_f64(a.table, 6);
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t t_begin = n_tiles * b / nb, t_end = n_tiles * (b + 1) / nb;

  auto load_ids = [&](int64_t t, uint32_t (&x)[kPcPPT], uint32_t (&y)[kPcPPT]) {
    const int64_t c0 = a.c_begin + t * kPcTile + int64_t(threadIdx.x) * kPcPPT;
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p) x[p] = y[p] = 0;
    if (KIND == BLSH_PAIRS && c0 + kPcPPT <= a.c_end && ((uintptr_t(a.x + c0) | uintptr_t(a.y + c0)) & 15) == 0) {
      const u32x4 vx = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.x + c0));
      const u32x4 vy = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.y + c0));
      x[0] = vx.x; x[1] = vx.y; x[2] = vx.z; x[3] = vx.w;
      y[0] = vy.x; y[1] = vy.y; y[2] = vy.z; y[3] = vy.w;
    } else {
#pragma unroll
      for (int p = 0; p < kPcPPT; ++p)
        if (c0 + p < a.c_end) fetch_candidate(a, c0 + p, x[p], y[p]);
    }
  };

  uint32_t nx[kPcPPT], ny[kPcPPT];
  if (t_begin < t_end) load_ids(t_begin, nx, ny);
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int64_t c0 = a.c_begin + t * kPcTile + int64_t(threadIdx.x) * kPcPPT;
    uint32_t xi[kPcPPT], yi[kPcPPT];
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p) { xi[p] = nx[p]; yi[p] = ny[p]; }
    uint32_t alive = 0, bad = 0;
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p) {
      if (c0 + p < a.c_end) {
        if (xi[p] < a.n_obj && yi[p] < a.n_obj) alive |= 1u << p; else bad |= 1u << p;
      }
    }
    // lookups
    uint32_t wx[kPcPPT][kPcWords], wy[kPcPPT][kPcWords];
    uint32_t miss_x = 0, miss_y = 0;
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p) {
      if (!(alive & (1u << p))) continue;
      const uint4 ux = s_slot[(xi[p] * 2654435761u) >> (32 - kPcSlotBits)];
      const uint4 uy = s_slot[(yi[p] * 2654435761u) >> (32 - kPcSlotBits)];
      if (ux.x == xi[p]) { wx[p][0] = ux.y; wx[p][1] = ux.z; wx[p][2] = ux.w; } else miss_x |= 1u << p;
      if (uy.x == yi[p]) { wy[p][0] = uy.y; wy[p][1] = uy.z; wy[p][2] = uy.w; } else miss_y |= 1u << p;
    }
    // misses gather the cached words from global memory
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p) {
#pragma unroll
      for (int w = 0; w < kPcWords; ++w) {
        if ((miss_x >> p) & 1u) wx[p][w] = w < cw ? sig_word<WM>(a, xi[p], w) : 0u;
        if ((miss_y >> p) & 1u) wy[p][w] = w < cw ? sig_word<WM>(a, yi[p], w) : 0u;
      }
    }
    // the next tile's ids are requested after this tile's gathers
    if (t + 1 < t_end) load_ids(t + 1, nx, ny);

    uint32_t m[kPcPPT] = {0, 0, 0, 0};
    uint8_t code[kPcPPT] = {0, 0, 0, 0};
    uint32_t emit = 0;
    for (int j = 0; j < L && alive; ++j) {
      const bool cached = level_first_word<K>(j) + level_words<K>(j) <= cw;
#pragma unroll
      for (int p = 0; p < kPcPPT; ++p) {
        if (!(alive & (1u << p))) continue;
        if (cached) {
          m[p] += agree_from<K>(wx[p], wy[p], j);
        } else {
          uint32_t gx[2], gy[2];
          const int f = level_first_word<K>(j);
          gx[0] = sig_word<WM>(a, xi[p], f);
          gy[0] = sig_word<WM>(a, yi[p], f);
          if (K == 64) { gx[1] = sig_word<WM>(a, xi[p], f + 1); gy[1] = sig_word<WM>(a, yi[p], f + 1); }
          else { gx[1] = gy[1] = 0u; }
          if constexpr (K == 32) m[p] += 32u - __popc(gx[0] ^ gy[0]);
          else if constexpr (K == 64) m[p] += 64u - __popc(gx[0] ^ gy[0]) - __popc(gx[1] ^ gy[1]);
          else m[p] += 16u - __popc(((gx[0] ^ gy[0]) >> ((j & 1) * 16)) & 0xFFFFu);
        }
        if (int(m[p]) < s_min[j]) {
          code[p] = uint8_t((BLSH_PRUNED << 6) | j);
          alive &= ~(1u << p);
        } else if (!LITE && accept_bit(a.table, words, j, int(m[p]))) {
          code[p] = uint8_t((BLSH_ACCEPT_CONC << 6) | j);
          alive &= ~(1u << p);
          emit |= 1u << p;
        } else if (j == L - 1) {
          code[p] = uint8_t(((LITE ? BLSH_LITE_EXACT : BLSH_ACCEPT_NMAX) << 6) | j);
          alive &= ~(1u << p);
          emit |= 1u << p;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p)
      if (bad & (1u << p)) code[p] = 0xFF;
    if (bad) raise_status(a.status, BLSH_EBADID);
    if (c0 < a.c_end) {
      if (c0 + kPcPPT <= a.c_end && (uintptr_t(a.code + c0) & 3) == 0) {
        const uint32_t packed = uint32_t(code[0]) | (uint32_t(code[1]) << 8) | (uint32_t(code[2]) << 16) |
                                (uint32_t(code[3]) << 24);
        __builtin_nontemporal_store(packed, reinterpret_cast<uint32_t *>(a.code + c0));
      } else {
#pragma unroll
        for (int p = 0; p < kPcPPT; ++p)
          if (c0 + p < a.c_end) a.code[c0 + p] = code[p];
      }
      if (a.m_dbg) {
#pragma unroll
        for (int p = 0; p < kPcPPT; ++p)
          if (c0 + p < a.c_end) a.m_dbg[c0 + p] = uint16_t(m[p]);
      }
    }
    if (__ballot(emit != 0) != 0) {
#pragma unroll
      for (int p = 0; p < kPcPPT; ++p) {
        const bool e = (emit >> p) & 1u;
        if (LITE) {
          push_survivor(a, e, c0 + p);
        } else {
          const int n = ((code[p] & 63) + 1) * K;
          const float v = e ? map_estimate(a.measure, int(m[p]), n, alpha, beta) : 0.f;
          emit_accepted(a, e, uint64_t(c0 + p), v);
        }
      }
    }
    // refill the slots of this tile's misses once every lookup of the tile is done
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kPcPPT; ++p) {
      if ((miss_x >> p) & 1u)
        s_slot[(xi[p] * 2654435761u) >> (32 - kPcSlotBits)] = make_uint4(xi[p], wx[p][0], wx[p][1], wx[p][2]);
      if ((miss_y >> p) & 1u)
        s_slot[(yi[p] * 2654435761u) >> (32 - kPcSlotBits)] = make_uint4(yi[p], wy[p][0], wy[p][1], wy[p][2]);
    }
    __syncthreads();
  }
}

template <int K, int KIND, bool LITE, bool WM>
static int launch_pc(const VerifyArgs &a, int n_cu, hipStream_t s) {
  const int64_t n = a.c_end - a.c_begin;
  const int64_t n_tiles = (n + kPcTile - 1) / kPcTile;
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(n_tiles, int64_t(n_cu) * 2));
  hipLaunchKernelGGL((k_verify_bits_pc<K, KIND, LITE, WM>), dim3(nb), dim3(kPcBlock), 0, s, a, n_tiles);
  return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
}

template <int K, bool LITE, bool WM>
static int launch_pc_kind(const VerifyArgs &a, int n_cu, hipStream_t s) {
  switch (a.kind) {
    case BLSH_PAIRS: return launch_pc<K, BLSH_PAIRS, LITE, WM>(a, n_cu, s);
    case BLSH_QUERY_LISTS: return launch_pc<K, BLSH_QUERY_LISTS, LITE, WM>(a, n_cu, s);
    default: return launch_pc<K, BLSH_ALL_PAIRS, LITE, WM>(a, n_cu, s);
  }
}

int launch_verify_bits_cached(blsh_ctx *ctx, const VerifyArgs &a, int k, bool lite, bool wm, hipStream_t s) {
  LaunchScope ls(ctx, s, "verify_bits_pcache");
#define BLSH_PC(KK, LL, WW) if (k == KK && lite == LL && wm == WW) return launch_pc_kind<KK, LL, WW>(a, ctx->n_cu, s);
  BLSH_PC(16, false, true) BLSH_PC(16, true, true) BLSH_PC(16, false, false) BLSH_PC(16, true, false)
  BLSH_PC(32, false, true) BLSH_PC(32, true, true) BLSH_PC(32, false, false) BLSH_PC(32, true, false)
  BLSH_PC(64, false, true) BLSH_PC(64, true, true) BLSH_PC(64, false, false) BLSH_PC(64, true, false)
#undef BLSH_PC
  return fail(BLSH_EINVAL, "unsupported k=%d", k);
}

}  // namespace blsh
