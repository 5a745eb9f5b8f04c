/* Plain C oracle loops for BayesLSH -- TEST INFRASTRUCTURE ONLY.
 *
 * Built by oracle/build.py with gcc into oracle/_build/liboracle.so and loaded
 * through ctypes by oracle/reference.py.  Nothing here is shared with the GPU
 * library.  Every loop is the literal per-item definition; there is no
 * blocking or vectorisation beyond an OpenMP loop over independent items.
 *
 *   philox4x32_10     counter-based generator of Salmon et al., "Parallel
 *                     random numbers: as easy as 1, 2, 3" (SC 2011),
 *                     Philox-4x32 with 10 rounds.
 *   srp_gauss         standard normal plane entry g(term, bit) for the sign
 *                     random projection family (Section 4.2): Box-Muller in
 *                     FP64 on two Philox words, rounded to float.
 *   srp_sparse_proj   r_b . x in FP64 for sparse rows (Section 4.2), optionally
 *                     with every plane entry stored in 2 bytes (Section 4.3).
 *   q16_encode/decode the 2-byte storage of a plane entry (Section 4.3).
 *   minhash           min over the set of (a_h e + b_h) mod (2^31-1)  (Section 4.1).
 *   verify            Algorithm 1 (BayesLSH) / Algorithm 2 (BayesLSH-Lite) per pair,
 *                     reading per-(m,n) decisions memoised by the Python oracle.
 *   mle               the classical estimator m/n over all hashes (Section 3).
 *   exact_*           exact cosine / Jaccard similarity (FP64).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- Philox4x32-10 ---------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Plane entry for hash `bit` and coordinate `term`:
 * counter (term, bit/4, 0, 0), key (seed low word, seed high word);
 * u_i = (w_i + 0.5) / 2^32; (z0,z1) = BoxMuller(u0,u1), (z2,z3) = BoxMuller(u2,u3);
 * the entry is z_{bit mod 4} rounded to float. */
float srp_gauss(uint64_t seed, uint32_t term, uint32_t bit) {
    uint32_t ctr[4] = {term, bit >> 2, 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    const double two32 = 4294967296.0;
    const double two_pi = 6.283185307179586476925286766559;
    int pair = (bit & 3u) >> 1;
    double u0 = ((double)w[2 * pair] + 0.5) / two32;
    double u1 = ((double)w[2 * pair + 1] + 0.5) / two32;
    double rho = sqrt(-2.0 * log(u0));
    double z = (bit & 1u) ? rho * sin(two_pi * u1) : rho * cos(two_pi * u1);
    return (float)z;
}

/* 2-byte storage of a Gaussian sample (Section 4.3, cheaper storage of hash
 * functions): x in (-8, 8) is kept as the integer floor((x + 8) 2^16 / 16);
 * values outside the interval saturate to the end codes.  The stored code is
 * read back as the midpoint of its interval of width 16 / 2^16, so the error
 * is at most half that width. */
uint16_t q16_encode(double x) {
    double c = floor((x + 8.0) * (65536.0 / 16.0));
    if (c < 0.0) c = 0.0;
    if (c > 65535.0) c = 65535.0;
    return (uint16_t)c;
}

double q16_decode(uint16_t code) {
    return ((double)code + 0.5) * (16.0 / 65536.0) - 8.0;
}

void q16_encode_array(const double *x, int64_t n, uint16_t *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = q16_encode(x[i]);
}

void q16_decode_array(const uint16_t *c, int64_t n, double *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = q16_decode(c[i]);
}

/* proj[r][b] = sum over the row's nonzeros of value * g(term, b), in FP64;
 * with q16 != 0 each entry g is replaced by its 2-byte code read back. */
void srp_sparse_proj(const int64_t *offsets, const uint32_t *indices, const float *values,
                     const int64_t *rows, int64_t n_rows, int32_t n_bits, uint64_t seed,
                     int32_t q16, double *proj) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = rows[r];
        for (int32_t b = 0; b < n_bits; ++b) {
            double acc = 0.0;
            for (int64_t e = offsets[i]; e < offsets[i + 1]; ++e) {
                double g = (double)srp_gauss(seed, indices[e], (uint32_t)b);
                if (q16) g = q16_decode(q16_encode(g));
                acc += (double)values[e] * g;
            }
            proj[r * (int64_t)n_bits + b] = acc;
        }
    }
}

/* ---------------- minhash ---------------- */
void minhash(const int64_t *offsets, const uint32_t *elems, const int64_t *rows, int64_t n_rows,
             const uint32_t *a, const uint32_t *b, int32_t n_hashes, uint32_t *out) {
    const uint64_t P = 2147483647ull;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t i = rows[r];
        for (int32_t h = 0; h < n_hashes; ++h) {
            uint64_t best = UINT64_MAX;
            for (int64_t e = offsets[i]; e < offsets[i + 1]; ++e) {
                uint64_t v = ((uint64_t)a[h] * (uint64_t)elems[e] + (uint64_t)b[h]) % P;
                if (v < best) best = v;
            }
            out[r * (int64_t)n_hashes + h] = (uint32_t)best;
        }
    }
}

/* ---------------- hash agreement ---------------- */
/* measure 0: sig rows of n_hashes uint32 (minhash); measure 1: rows of n_hashes/32
 * packed words, hash i = bit (i mod 32) of word i/32. */
static int agree(int measure, const uint32_t *sx, const uint32_t *sy, int32_t i) {
    if (measure == 0) return sx[i] == sy[i];
    uint32_t bx = (sx[i >> 5] >> (i & 31)) & 1u;
    uint32_t by = (sy[i >> 5] >> (i & 31)) & 1u;
    return bx == by;
}

enum { DEC_PRUNED = 0, DEC_CONC = 1, DEC_NMAX = 2, DEC_LITE = 3 };

/* One pair through Algorithm 1 (lite = 0) or Algorithm 2 (lite = 1).
 * survive/accept are [n_levels][n_max+1] byte tables of the per-(m,n)
 * decisions; level j covers hashes [j k, (j+1) k). */
static void run_pair(int measure, const uint32_t *sx, const uint32_t *sy, int32_t k, int32_t n_levels,
                     int32_t n_max, int lite, const uint8_t *survive, const uint8_t *accept,
                     uint8_t *dec, int16_t *lvl_out, int32_t *m_out) {
    int32_t n = 0, m = 0;
    for (int32_t j = 0; j < n_levels; ++j) {
        for (int32_t i = n; i < n + k; ++i) m += agree(measure, sx, sy, i);
        n += k;
        const int64_t at = (int64_t)j * (n_max + 1) + m;
        if (!survive[at]) { *dec = DEC_PRUNED; *lvl_out = (int16_t)j; *m_out = m; return; }
        if (!lite && accept[at]) { *dec = DEC_CONC; *lvl_out = (int16_t)j; *m_out = m; return; }
    }
    *dec = lite ? DEC_LITE : DEC_NMAX;
    *lvl_out = (int16_t)(n_levels - 1);
    *m_out = m;
}

/* kind 0: explicit pairs (x[p], y[p]); kind 2: all pairs i < j of [0, all_n), row-major. */
void verify(int32_t kind, const uint32_t *x, const uint32_t *y, int64_t n_pairs, int64_t all_n,
            int32_t measure, const uint32_t *sig, int32_t row_words, int32_t k, int32_t n_levels,
            int32_t lite, const uint8_t *survive, const uint8_t *accept,
            uint8_t *dec, int16_t *lvl, int32_t *mm) {
    const int32_t n_max = k * n_levels;
    if (kind == 0) {
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t p = 0; p < n_pairs; ++p)
            run_pair(measure, sig + (int64_t)x[p] * row_words, sig + (int64_t)y[p] * row_words, k, n_levels,
                     n_max, lite, survive, accept, dec + p, lvl + p, mm + p);
    } else {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t i = 0; i < all_n; ++i) {
            int64_t p = i * all_n - i * (i + 1) / 2;
            for (int64_t j = i + 1; j < all_n; ++j, ++p)
                run_pair(measure, sig + i * row_words, sig + j * row_words, k, n_levels, n_max, lite,
                         survive, accept, dec + p, lvl + p, mm + p);
        }
    }
}

/* Classical estimate over the first n_hashes hashes: m_total per pair. */
void count_all(const uint32_t *x, const uint32_t *y, int64_t n_pairs, int32_t measure,
               const uint32_t *sig, int32_t row_words, int32_t n_hashes, int32_t *m_out) {
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t p = 0; p < n_pairs; ++p) {
        const uint32_t *sx = sig + (int64_t)x[p] * row_words, *sy = sig + (int64_t)y[p] * row_words;
        int32_t m = 0;
        for (int32_t i = 0; i < n_hashes; ++i) m += agree(measure, sx, sy, i);
        m_out[p] = m;
    }
}

/* ---------------- exact similarity ---------------- */
/* cosine of sparse rows with sorted indices: dot / (|x| |y|), all sums in FP64. */
void exact_cosine_csr(const int64_t *offsets, const uint32_t *indices, const float *values,
                      const uint32_t *x, const uint32_t *y, int64_t n, double *out) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < n; ++p) {
        int64_t a = offsets[x[p]], ae = offsets[x[p] + 1];
        int64_t b = offsets[y[p]], be = offsets[y[p] + 1];
        double nx = 0.0, ny = 0.0, dot = 0.0;
        for (int64_t e = a; e < ae; ++e) nx += (double)values[e] * (double)values[e];
        for (int64_t e = b; e < be; ++e) ny += (double)values[e] * (double)values[e];
        while (a < ae && b < be) {
            if (indices[a] == indices[b]) { dot += (double)values[a] * (double)values[b]; ++a; ++b; }
            else if (indices[a] < indices[b]) ++a;
            else ++b;
        }
        out[p] = (nx > 0.0 && ny > 0.0) ? dot / (sqrt(nx) * sqrt(ny)) : 0.0;
    }
}

void exact_cosine_dense(const float *X, int64_t d, const uint32_t *x, const uint32_t *y, int64_t n,
                        double *out) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < n; ++p) {
        const float *u = X + (int64_t)x[p] * d, *v = X + (int64_t)y[p] * d;
        double nx = 0.0, ny = 0.0, dot = 0.0;
        for (int64_t c = 0; c < d; ++c) {
            nx += (double)u[c] * (double)u[c];
            ny += (double)v[c] * (double)v[c];
            dot += (double)u[c] * (double)v[c];
        }
        out[p] = (nx > 0.0 && ny > 0.0) ? dot / (sqrt(nx) * sqrt(ny)) : 0.0;
    }
}

/* Jaccard of sorted sets: |A n B| / |A u B|. */
void exact_jaccard(const int64_t *offsets, const uint32_t *elems, const uint32_t *x, const uint32_t *y,
                   int64_t n, double *out) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < n; ++p) {
        int64_t a = offsets[x[p]], ae = offsets[x[p] + 1];
        int64_t b = offsets[y[p]], be = offsets[y[p] + 1];
        int64_t inter = 0, na = ae - a, nb = be - b;
        while (a < ae && b < be) {
            if (elems[a] == elems[b]) { ++inter; ++a; ++b; }
            else if (elems[a] < elems[b]) ++a;
            else ++b;
        }
        int64_t uni = na + nb - inter;
        out[p] = uni > 0 ? (double)inter / (double)uni : 0.0;
    }
}
