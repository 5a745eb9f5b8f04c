// Signature generation kernels for gfx950 (Section 4 LSH families).
//
//   k_minhash          one wave per set, lanes over hash functions; each lane keeps
//                      the running minimum of (a_h e + b_h) mod (2^31 - 1) over the
//                      set's elements (Section 4.1).
//   k_srp_sparse       one wave per sparse row, lanes over groups of 4 hashes; plane
//                      entries come from Philox-4x32-10 + Box-Muller (FP64), the
//                      projections accumulate in FP64, and the sign bits are packed
//                      32 to a word with DPP (Section 4.2).  Optionally every entry
//                      is stored in 2 bytes (Section 4.3): a table of codes then
//                      takes half the bytes of the fp32 one.
//   k_srp_dense_mfma   dense rows times a Gaussian plane matrix on the matrix cores
//                      (v_mfma_f32_32x32x2f32); each wave keeps 32 rows of X in
//                      registers, the block stages a 32-plane slice of R in LDS, and
//                      the sign of every accumulator is packed with a wave ballot.
#include <type_traits>

#include "device_common.h"

namespace blsh {

// ---------------------------------------------------------------------------
// Minhash
// ---------------------------------------------------------------------------
template <int HPL>  // hashes per lane
__global__ __launch_bounds__(256) void k_minhash(const int64_t *offsets, const uint32_t *elems, int64_t n_sets,
                                                 const uint32_t *a, const uint32_t *b, int32_t n_hashes,
                                                 uint32_t *out, int32_t *status) {
  const int lane = lane_id();
  const int64_t set = __builtin_amdgcn_readfirstlane(int(blockIdx.x)) * int64_t(4) + (threadIdx.x >> 6);
  if (set >= n_sets) return;
  constexpr uint64_t P = 2147483647ull;
  uint64_t ah[HPL], bh[HPL];
  uint32_t best[HPL];
#pragma unroll
  for (int i = 0; i < HPL; ++i) {
    const int h = lane + kWave * i;
    ah[i] = h < n_hashes ? a[h] : 0;
    bh[i] = h < n_hashes ? b[h] : 0;
    best[i] = 0xFFFFFFFFu;
  }
  const int64_t s = offsets[set], e = offsets[set + 1];
  if (e <= s) raise_status(status, BLSH_EINVAL);
  for (int64_t q = s; q < e; ++q) {
    const uint64_t el = elems[q];
#pragma unroll
    for (int i = 0; i < HPL; ++i) {
      uint64_t v = ah[i] * el + bh[i];
      v = (v & P) + (v >> 31);
      v = (v & P) + (v >> 31);
      if (v >= P) v -= P;
      best[i] = min(best[i], uint32_t(v));
    }
  }
#pragma unroll
  for (int i = 0; i < HPL; ++i) {
    const int h = lane + kWave * i;
    if (h < n_hashes) out[size_t(set) * n_hashes + h] = best[i];
  }
}

// ---------------------------------------------------------------------------
// Philox-4x32-10 (Salmon et al., SC 2011) and the plane entries
// ---------------------------------------------------------------------------
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// The four plane entries for hashes 4q..4q+3 at coordinate `term`.
__device__ inline void srp_gauss4(uint32_t term, uint32_t q, uint32_t k0, uint32_t k1, double g[4]) {
  const uint4 w = philox4x32_10(make_uint4(term, q, 0u, 0u), k0, k1);
  const double two32 = 4294967296.0, two_pi = 6.283185307179586476925286766559;
  const double u0 = (double(w.x) + 0.5) / two32, u1 = (double(w.y) + 0.5) / two32;
  const double u2 = (double(w.z) + 0.5) / two32, u3 = (double(w.w) + 0.5) / two32;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  double s1, c1, s3, c3;   // one argument reduction for each sine-cosine pair
  sincos(two_pi * u1, &s1, &c1);
  sincos(two_pi * u3, &s3, &c3);
  g[0] = double(float(r0 * c1));
  g[1] = double(float(r0 * s1));
  g[2] = double(float(r1 * c3));
  g[3] = double(float(r1 * s3));
}

// 2-byte storage of a plane entry (Section 4.3): g in (-8, 8) becomes the
// integer floor((g + 8) 2^16 / 16), saturating outside; the code is read back
// as the middle of its cell of width 2^-12 (error at most 2^-13).  Both steps
// are exact in FP64 for every fp32 entry.
__device__ inline uint32_t q16_code(double g) {
  const double c = floor((g + 8.0) * 4096.0);
  return uint32_t(fmin(fmax(c, 0.0), 65535.0));
}

__device__ inline double q16_value(uint32_t code) { return (double(code) + 0.5) * (1.0 / 4096.0) - 8.0; }

template <int G>
__device__ inline uint32_t group_or(uint32_t v) {
  if constexpr (G >= 2) v |= dpp<kDppQuadXor1>(v);
  if constexpr (G >= 4) v |= dpp<kDppQuadXor2>(v);
  if constexpr (G >= 8) v |= dpp<kDppHalfMirror>(v);
  return v;
}

// used[term] = 1 for every term < dim that some nonzero holds (used[] zeroed
// before).
__global__ __launch_bounds__(256) void k_srp_mark(const uint32_t *indices, int64_t nnz, int64_t dim,
                                                  uint8_t *used) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nnz; i += int64_t(gridDim.x) * 256) {
    const uint32_t t = indices[i];
    if (int64_t(t) < dim) used[t] = 1;
  }
}

__global__ __launch_bounds__(256) void k_fill_u8(uint8_t *p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) p[i] = 0;
}

// Plane entries of the terms < dim that occur (used[term] != 0),
// table[term][n_bits] of fp32 (Q16: of 2-byte codes): one thread per (term,
// quad of hashes).  Used when each term occurs in several rows, so that an
// entry is drawn once instead of once per occurrence.
template <bool Q16>
__global__ __launch_bounds__(256) void k_srp_table(int64_t dim, int32_t n_bits, uint32_t k0, uint32_t k1,
                                                   const uint8_t *used, void *table) {
  const int Q = n_bits / 4;
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= dim * Q) return;
  const int64_t term = i / Q;
  if (!used[term]) return;
  const int q = int(i % Q);
  double g[4];
  srp_gauss4(uint32_t(term), uint32_t(q), k0, k1, g);
  const size_t at = size_t(term) * n_bits + 4 * q;
  if constexpr (Q16) {
    const uint2 w = make_uint2(q16_code(g[0]) | q16_code(g[1]) << 16, q16_code(g[2]) | q16_code(g[3]) << 16);
    *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(table) + at) = w;
  } else {
    *reinterpret_cast<float4 *>(static_cast<float *>(table) + at) =
        make_float4(float(g[0]), float(g[1]), float(g[2]), float(g[3]));
  }
}

// The four entries of hashes 4q..4q+3 at `term`, read from the table row or
// drawn (terms >= dim); Q16: as their 2-byte codes read back.
template <bool Q16>
__device__ inline void srp_entry4(const void *table, int64_t dim, int32_t n_bits, uint32_t term, int q, uint32_t k0,
                                  uint32_t k1, double g[4]) {
  srp_gauss4(term, uint32_t(q), k0, k1, g);
  if constexpr (Q16) {
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = q16_value(q16_code(g[c]));
  }
  (void)table; (void)dim; (void)n_bits;
}

// TABLE: entries of terms < dim come from the table (the same values the
// generator gives, since every entry is rounded to fp32, or the same codes),
// others are drawn.  Q16: every entry is the value its 2-byte code stands for.
// With a table the row's nonzeros are taken U at a time: the U table rows are
// requested before any is used, so that U dependent fetches overlap (a batch
// with a term outside the table leaves the rest of the row to the loop that
// takes one nonzero at a time).
// A wave takes one row and 64 QPL consecutive quads of its hashes (a slice;
// rows of more hashes take several waves).
template <int QPL, bool TABLE, bool Q16>  // quads (4 hashes) per lane
__global__ __launch_bounds__(256) void k_srp_sparse(const int64_t *offsets, const uint32_t *indices,
                                                    const float *values, int64_t n_rows, int32_t n_bits,
                                                    int32_t n_slices, uint32_t k0, uint32_t k1, int32_t word_major,
                                                    uint32_t *out, const void *table, int64_t dim) {
  constexpr int U = TABLE ? (Q16 ? 4 : 2) : 1;
  using Entry = typename std::conditional<Q16, uint2, float4>::type;
  const int lane = lane_id();
  const int64_t wid = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t row = wid / n_slices;
  if (row >= n_rows) return;  // wave-uniform
  const int q0 = int(wid % n_slices) * kWave * QPL;   // first quad of the slice
  const int Q = n_bits / 4, W = n_bits / 32;
  double acc[QPL][4];
#pragma unroll
  for (int i = 0; i < QPL; ++i)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[i][c] = 0.0;
  const int64_t s = offsets[row], e = offsets[row + 1];
  auto fma4 = [&](int i, double v, const double g[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[i][c] += v * g[c];
  };
  auto decode = [&](const Entry &x, double g[4]) {
    if constexpr (Q16) {
      g[0] = q16_value(x.x & 0xFFFFu); g[1] = q16_value(x.x >> 16);
      g[2] = q16_value(x.y & 0xFFFFu); g[3] = q16_value(x.y >> 16);
    } else {
      g[0] = x.x; g[1] = x.y; g[2] = x.z; g[3] = x.w;
    }
  };
  int64_t t = s;
  if constexpr (TABLE) {
    for (; t + U <= e; t += U) {
      uint32_t term[U];
      double v[U];
      bool in_table = true;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        term[u] = indices[t + u];
        v[u] = values[t + u];
        in_table = in_table && int64_t(term[u]) < dim;
      }
      if (!in_table) break;   // a term outside the table: the rest of the row one nonzero at a time
      Entry ent[U][QPL];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
          const int q = q0 + lane + kWave * i;
          if (q < Q)
            ent[u][i] = *reinterpret_cast<const Entry *>(static_cast<const typename std::conditional<
                            Q16, uint16_t, float>::type *>(table) + size_t(term[u]) * n_bits + 4 * q);
        }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < QPL; ++i) {
          const int q = q0 + lane + kWave * i;
          if (q < Q) {
            double g[4];
            decode(ent[u][i], g);
            fma4(i, v[u], g);
          }
        }
    }
  }
  for (; t < e; ++t) {
    const uint32_t term = indices[t];
    const double v = values[t];
#pragma unroll
    for (int i = 0; i < QPL; ++i) {
      const int q = q0 + lane + kWave * i;
      if (q < Q) {
        double g[4];
        if (TABLE && int64_t(term) < dim) {
          decode(*reinterpret_cast<const Entry *>(static_cast<const typename std::conditional<
                     Q16, uint16_t, float>::type *>(table) + size_t(term) * n_bits + 4 * q), g);
        } else {
          srp_entry4<Q16>(table, dim, n_bits, term, q, k0, k1, g);
        }
        fma4(i, v, g);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < QPL; ++i) {
    const int q = q0 + lane + kWave * i;
    uint32_t nib = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) nib |= uint32_t(acc[i][c] >= 0.0) << c;
    uint32_t word = group_or<8>(q < Q ? nib << (4 * (lane & 7)) : 0u);
    const int w = q >> 3;
    if ((lane & 7) == 0 && w < W) {
      if (word_major) out[size_t(w) * n_rows + row] = word;
      else out[size_t(row) * W + w] = word;
    }
  }
}

// ---------------------------------------------------------------------------
// Dense SRP on the matrix cores
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));

// X: [n_rows][D] fp32, R: [D][n_bits] fp32.  Block = 4 waves = 128 rows; the
// D dimension is split between the two half-waves: lanes 0..31 cover
// d in [0, D/2) and lanes 32..63 cover [D/2, D), so that each lane's A
// operands are one contiguous half-row of X.  The 32-plane slices of R are
// double-buffered in LDS: the next slice is read into registers before the
// current one's MFMA loop and written to the other buffer after it, so one
// barrier per slice remains and the reads overlap the matrix work.
template <int D>
__global__ __launch_bounds__(256, 2) void k_srp_dense_mfma(const float *X, int64_t n_rows, const float *R,
                                                        int32_t n_bits, int32_t word_major, uint32_t *out) {
  constexpr int HD = D / 2;
  constexpr int PER = D * 32 / 256;   // slice entries per thread
  __shared__ float sR[2][D * 32];     // 32-plane slices: sR[b][d*32 + j] = R[d][col0 + j]
  const int lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const int h = lane >> 5, i = lane & 31;
  const int64_t row0 = int64_t(blockIdx.x) * 128 + wv * 32;
  const int64_t my_row = row0 + i;
  float xa[HD];
  if (my_row < n_rows) {
    const float4 *src = reinterpret_cast<const float4 *>(X + size_t(my_row) * D + h * HD);
#pragma unroll
    for (int q = 0; q < HD / 4; ++q) {
      const float4 v = src[q];
      xa[4 * q] = v.x; xa[4 * q + 1] = v.y; xa[4 * q + 2] = v.z; xa[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < HD; ++q) xa[q] = 0.f;
  }
  const int W = n_bits / 32;
  // row held in the result word by this lane (lanes 0..31): t = lane
  const int t = lane & 31;
  const int my_v = 4 * (t >> 3) + (t & 3), my_h = (t >> 2) & 1;
  float st[PER];
  auto fetch = [&](int tile) {   // entry idx = threadIdx.x + 256 u of the slice: d = idx / 32, j = idx % 32
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int idx = int(threadIdx.x) + 256 * u;
      st[u] = R[size_t(idx >> 5) * n_bits + tile * 32 + (idx & 31)];
    }
  };
  auto stash = [&](int b) {
#pragma unroll
    for (int u = 0; u < PER; ++u) sR[b][int(threadIdx.x) + 256 * u] = st[u];
  };
  fetch(0);
  stash(0);
  __syncthreads();
  for (int tile = 0; tile < W; ++tile) {
    const int b = tile & 1;
    if (tile + 1 < W) fetch(tile + 1);
    floatx16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < HD; ++s) {
      const float bv = sR[b][(h * HD + s) * 32 + i];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[s], bv, acc, 0, 0, 0);
    }
    uint32_t word = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const uint64_t mk = __ballot(acc[v] >= 0.f);
      if (my_v == v) word = my_h ? uint32_t(mk >> 32) : uint32_t(mk);
    }
    const int64_t r = row0 + t;
    if (lane < 32 && r < n_rows) {
      if (word_major) out[size_t(tile) * n_rows + r] = word;
      else out[size_t(r) * W + tile] = word;
    }
    // buffer b ^ 1 was last read in the previous slice, before the barrier
    // that ended it; the barrier below orders these writes before its reads
    if (tile + 1 < W) stash(b ^ 1);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int launch_minhash(blsh_ctx *ctx, const int64_t *offsets, const uint32_t *elems, int64_t n_sets, const uint32_t *a,
                   const uint32_t *b, int n_hashes, uint32_t *out, hipStream_t s) {
  const int hpl = (n_hashes + kWave - 1) / kWave;
  const int64_t nb = (n_sets + 3) / 4;
  LaunchScope ls(ctx, s, "minhash_sigs");
#define BLSH_MH(N) if (hpl <= N) { hipLaunchKernelGGL(k_minhash<N>, dim3(nb), dim3(256), 0, s, offsets, elems, n_sets, a, b, n_hashes, out, ctx->d_status); return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE; }
  BLSH_MH(1) BLSH_MH(2) BLSH_MH(4) BLSH_MH(8) BLSH_MH(16)
#undef BLSH_MH
  return fail(BLSH_EINVAL, "minhash: n_hashes %d > 1024", n_hashes);
}

constexpr size_t kSrpTableMaxBytes = size_t(16) << 30;

int launch_srp_sparse(blsh_ctx *ctx, const int64_t *offsets, const uint32_t *indices, const float *values,
                      int64_t n_rows, int64_t dim, int n_bits, uint64_t seed, bool word_major, bool q16,
                      uint32_t *out, hipStream_t s) {
  // quads per lane: up to 4 (1024 hashes per wave); longer rows in slices of 1024
  const int quads = n_bits / 4;
  const int qpl_all = (quads + kWave - 1) / kWave;
  if (qpl_all > 8) return fail(BLSH_EINVAL, "srp (sparse): n_bits %d > 2048", n_bits);
  const int qpl = std::min(qpl_all, 4);
  const int n_slices = (qpl_all + qpl - 1) / qpl;
  const int64_t nb = (n_rows * n_slices + 3) / 4;
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  // a table of plane entries pays when terms repeat: more nonzeros than twice the dimension
  int64_t nnz = 0;
  BLSH_HIP(hipMemcpyAsync(&nnz, offsets + n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BLSH_HIP(hipStreamSynchronize(s));
  const size_t entry_bytes = q16 ? sizeof(uint16_t) : sizeof(float);
  const size_t table_bytes = size_t(std::max<int64_t>(dim, 0)) * size_t(n_bits) * entry_bytes;
  // (a context whose workspace is fixed too small for the table draws the
  // entries per nonzero instead: the same values)
  const bool use_table = dim > 0 && nnz > 2 * dim && table_bytes <= kSrpTableMaxBytes &&
                         (!ctx->ws_fixed || table_bytes + size_t(dim) <= ctx->ws_bytes);
  void *table = nullptr;
  uint8_t *used = nullptr;   // one byte per term after the table
  if (use_table) {
    if (int rc = ensure_workspace(ctx, table_bytes + size_t(dim))) return rc;
    table = ctx->ws;
    used = static_cast<uint8_t *>(ctx->ws) + table_bytes;
  }
  LaunchScope ls(ctx, s, "srp_sparse");
  if (use_table) {
    // draw the entries of the terms that occur
    const unsigned gz = unsigned(std::min<int64_t>((dim + 255) / 256, 4096));
    hipLaunchKernelGGL(k_fill_u8, dim3(gz), dim3(256), 0, s, used, dim);
    const unsigned gm = unsigned(std::min<int64_t>((nnz + 255) / 256, 8192));
    hipLaunchKernelGGL(k_srp_mark, dim3(gm), dim3(256), 0, s, indices, nnz, dim, used);
    const int64_t items = dim * (n_bits / 4);
    const dim3 g(unsigned((items + 255) / 256));
    if (q16) hipLaunchKernelGGL(k_srp_table<true>, g, dim3(256), 0, s, dim, n_bits, k0, k1, used, table);
    else hipLaunchKernelGGL(k_srp_table<false>, g, dim3(256), 0, s, dim, n_bits, k0, k1, used, table);
  }
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nb), dim3(256), 0, s, offsets, indices, values, n_rows, n_bits, n_slices, k0, k1,
                       int(word_major), out, static_cast<const void *>(table), dim);
    return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE;
  };
#define BLSH_SP(N)                                                           \
  if (qpl <= N) {                                                            \
    if (use_table) return q16 ? go(k_srp_sparse<N, true, true>) : go(k_srp_sparse<N, true, false>); \
    return q16 ? go(k_srp_sparse<N, false, true>) : go(k_srp_sparse<N, false, false>);              \
  }
  BLSH_SP(1) BLSH_SP(2) BLSH_SP(4)
#undef BLSH_SP
  return fail(BLSH_EINVAL, "srp (sparse): n_bits %d > 2048", n_bits);
}

int launch_srp_dense(blsh_ctx *ctx, const float *X, int64_t n_rows, int64_t dim, const float *R, int n_bits,
                     bool word_major, uint32_t *out, hipStream_t s) {
  const int64_t nb = (n_rows + 127) / 128;
  LaunchScope ls(ctx, s, "srp_dense_mfma");
#define BLSH_DN(DD) if (dim == DD) { hipLaunchKernelGGL(k_srp_dense_mfma<DD>, dim3(nb), dim3(256), 0, s, X, n_rows, R, n_bits, int(word_major), out); return hipGetLastError() == hipSuccess ? BLSH_OK : BLSH_EDEVICE; }
  BLSH_DN(32) BLSH_DN(64) BLSH_DN(128) BLSH_DN(256)
#undef BLSH_DN
  return fail(BLSH_EINVAL, "srp (dense): dim must be 32, 64, 128 or 256 (got %lld)", (long long)dim);
}

}  // namespace blsh
