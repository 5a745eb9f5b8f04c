/* bayeslsh.h -- C ABI of libbayeslsh.so, BayesLSH candidate verification on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow Satuluri & Parthasarathy, "Bayesian Locality Sensitive
 * Hashing for Fast Similarity Search":
 *   - the problem statement and output guarantees (Section 1),
 *   - Algorithm 1 (BayesLSH: prune, else estimate until concentrated) and
 *     Algorithm 2 (BayesLSH-Lite: prune with at most h hashes, then exact
 *     similarity) of Section 4,
 *   - the Jaccard (minhash, Beta prior; Section 4.1) and cosine (sign random
 *     projections, uniform prior on r; Section 4.2) instantiations,
 *   - the precomputation of minimum matches and the cache of concentration
 *     decisions (Section 4.3).
 *
 * Conventions shared by every call
 *   - Pointers are DEVICE pointers unless their name ends in _host.  The
 *     caller owns all input and output memory.
 *   - Calls that take `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream) only enqueue work and return; bayeslsh_sync() waits and
 *     reports errors the kernels raised.
 *   - Every call returns a blsh_status.  Nothing is thrown or aborted across
 *     the ABI; on failure bayeslsh_last_error() returns a thread-local message.
 *   - Arguments are validated on the host before anything is enqueued; an
 *     invalid call enqueues nothing and leaves outputs untouched.
 *   - A context (blsh_ctx) belongs to one device.  Calls on one context from
 *     several host threads must be serialised by the caller.  Calls on
 *     different streams of one context may overlap on the device only if
 *     they do not share output buffers; they share the context's workspace
 *     only through per-call slices, so overlapping calls must use separate
 *     contexts.
 */
#ifndef BAYESLSH_H
#define BAYESLSH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BAYESLSH_VERSION 4

typedef enum {
  BLSH_OK = 0,
  BLSH_EINVAL = -1,      /* invalid argument (shape, range, null pointer, layout) */
  BLSH_ENOMEM = -2,      /* device allocation failed or workspace too small */
  BLSH_EDEVICE = -3,     /* a HIP runtime call failed */
  BLSH_ETRUNCATED = -4,  /* the accepted list overflowed acc_capacity (n_accepted holds the true count) */
  BLSH_EBADID = -5,      /* a candidate referenced an object id >= n_obj (code byte 0xFF for that candidate) */
  BLSH_EAGAIN = 1        /* serving: request not finished yet */
} blsh_status;

/* Similarity measures (Section 4). */
typedef enum { BLSH_JACCARD = 0, BLSH_COSINE = 1 } blsh_measure;

/* Per-candidate decision, stored in bits 7..6 of the code byte; bits 5..0 hold
 * the level j at which the decision was taken (n = (j+1) k hashes compared).
 * Code 0xFF marks a candidate with an out-of-range object id. */
typedef enum {
  BLSH_PRUNED = 0,       /* Pr[S >= t | M(m,n)] < epsilon                      (Alg. 1/2) */
  BLSH_ACCEPT_CONC = 1,  /* Pr[|S - S_hat| < delta | M(m,n)] >= 1 - gamma      (Alg. 1)   */
  BLSH_ACCEPT_NMAX = 2,  /* undecided when the signature ran out (n = n_max)   (Alg. 1)   */
  BLSH_LITE_EXACT = 3    /* survived h hashes; exact similarity computed        (Alg. 2)   */
} blsh_decision;

/* Signature layouts. */
typedef enum {
  BLSH_OBJECT_MAJOR = 0, /* row per object: minhash uint32[n_obj][n_hashes];
                            SRP uint32[n_obj][n_hashes/32] packed bits          */
  BLSH_WORD_MAJOR = 1    /* SRP only: uint32[n_hashes/32][n_obj]; word w of all
                            objects is contiguous (level-major slabs)          */
} blsh_layout;

/* Candidate kinds (Alg. 1/2 input C). */
typedef enum {
  BLSH_PAIRS = 0,        /* candidate c = (x[c], y[c]), c in [0, n_pairs)                    */
  BLSH_QUERY_LISTS = 1,  /* list l = (query[l], cand[offsets[l] .. offsets[l+1])); candidate
                            index c = position in cand                                       */
  BLSH_ALL_PAIRS = 2,    /* all i < j over [0, all_n), row-major: c = i*all_n - i(i+1)/2 + j-i-1 */
  BLSH_TILES = 3         /* LSH buckets as 16 x 16 tiles of member pairs (bayeslsh_band_tiles): tile t's
                            candidates are numbered from tiles[t].first, see blsh_tile                */
} blsh_cand_kind;

/* One 16 x 16 tile of an LSH bucket's member pairs (Section 2 banding, written
 * by bayeslsh_band_tiles).  Position p = 16 r + c (r, c in [0, 16)) stands for
 * the pair (ids[r], ids[16 + c]): row r's member and column c's member; it is
 * a candidate iff bit p % 64 of keep[p / 64] is set, and the candidates of the
 * tile are numbered first, first + 1, ... in increasing p.  192 bytes. */
typedef struct {
  int64_t first;           /* candidate index of the tile's first candidate         */
  uint32_t n_rows, n_cols; /* members on the tile's rows / columns, 1..16           */
  uint64_t keep[4];        /* the candidate positions (row-major bit mask)          */
  uint32_t ids[32];        /* object ids: rows 0..15, then columns 0..15            */
  uint32_t reserved[4];
} blsh_tile;

/* Vector kinds for exact similarity (Alg. 2) and signature generation. */
typedef enum {
  BLSH_DENSE = 0,        /* float dense[n_obj][dim], row-major                       */
  BLSH_CSR = 1,          /* float values + uint32 indices (sorted, unique per row)   */
  BLSH_SETS = 2          /* uint32 indices only (sorted, unique per row): binary sets */
} blsh_vec_kind;

/* Prior (Section 4.1: Beta(alpha, beta) for Jaccard; Section 4.2: uniform on
 * r in [0.5, 1] for cosine).  Jaccard: 0 < alpha, beta <= 1e6 (integers use
 * the exact Beta-binomial closed form, other values the continued fraction of
 * the incomplete beta; see bayeslsh_fit_prior).  Cosine: must be {1, 1}. */
typedef struct { double alpha, beta; } blsh_prior;

typedef struct {
  blsh_measure measure;
  blsh_layout layout;
  const uint32_t *data;
  int64_t n_obj;
  int32_t n_hashes;      /* hashes stored per object (SRP: multiple of 32)            */
  int32_t n_max;         /* hashes verification may use, 0 = n_hashes; multiple of k   */
  const uint32_t *prefix; /* SRP, optional (NULL = none): hashes 0..127 of every object
                             again, object-major, 4 words per object, 16-byte aligned
                             (n_hashes >= 128).  The verification kernels then read a
                             candidate's first 128 hashes with one 16-byte gather from
                             this 16 B/object array, and later hashes from `data`.  The
                             caller keeps it equal to the first 128 hashes of `data`
                             (bayeslsh_srp_sigs with n_bits = 128 and the same seed or
                             the first 128 plane columns writes it).                  */
} blsh_sigs;

typedef struct {
  blsh_cand_kind kind;
  const uint32_t *x, *y;         /* PAIRS                     */
  int64_t n_pairs;
  const uint32_t *query;         /* QUERY_LISTS: [n_lists]     */
  const int64_t *offsets;        /* QUERY_LISTS: [n_lists + 1] */
  const uint32_t *cand;          /* QUERY_LISTS: [offsets[n_lists]] */
  int64_t n_lists;
  int64_t n_cand;                /* QUERY_LISTS: offsets[n_lists] (host copy of the total);
                                    TILES: the number of candidates the tiles hold */
  int64_t all_n;                 /* ALL_PAIRS                 */
  const blsh_tile *tiles;        /* TILES: [n_tiles], 16-byte aligned */
  int64_t n_tiles;
} blsh_candidates;

typedef struct {
  blsh_vec_kind kind;
  int64_t n_obj;
  int64_t dim;                   /* DENSE: columns; CSR/SETS: index bound (indices < dim) */
  const float *dense;            /* DENSE                     */
  const int64_t *offsets;        /* CSR/SETS: [n_obj + 1]      */
  const uint32_t *indices;       /* CSR/SETS                   */
  const float *values;           /* CSR                        */
} blsh_vectors;

/* Outputs of a verification call.  Every field except m_debug is required.
 *   code[c]      decision << 6 | level, one byte per candidate (fully overwritten)
 *   acc_idx/val  the output set O, compacted in unspecified order: candidate
 *                index and S_hat (Alg. 1) or the exact similarity (Alg. 2), fp32
 *   n_accepted   device int64: true size of O even when it exceeds acc_capacity
 *   m_debug      optional uint16 per candidate: m when the decision was taken */
typedef struct {
  uint8_t *code;
  uint64_t *acc_idx;
  float *acc_val;
  int64_t acc_capacity;
  int64_t *n_accepted;
  uint16_t *m_debug;
} blsh_result;

typedef struct blsh_ctx blsh_ctx;

/* ---------------- context ---------------- */

/* Create a context on HIP device `device`.  The context owns the posterior
 * table cache (host and device copies), a survivor workspace that grows on
 * demand (the growth synchronises the device) and the counters of the
 * accepted-pair staging.  Calls on one context share these: calls that may
 * run at the same time on the device (different streams) need different
 * contexts; calls queued on one stream are fine.  Returns BLSH_EDEVICE if the
 * device is absent. */
int bayeslsh_create(blsh_ctx **out, int device);
void bayeslsh_destroy(blsh_ctx *ctx);

/* Caller control of the context workspace (the device memory that
 * verification, Lite, the comparator, banding and the sparse SRP plane table
 * use beyond the caller's inputs and outputs).  bayeslsh_reserve_workspace
 * makes it at least `bytes` now (allocating synchronises the device once).
 * With fixed != 0 later calls never grow it: a call that needs more returns
 * BLSH_ENOMEM before launching any kernel or writing any output (a table
 * image may already have been uploaded to the cache), and the sparse SRP draws its plane
 * entries per nonzero instead of building a table that does not fit (the
 * same signatures).  fixed = 0 restores growth on demand.  A caller that
 * wants no allocation after setup runs its largest call once, reads the size
 * with bayeslsh_workspace_bytes and reserves it fixed.  The batched state,
 * the banding tile buffer and the posterior-table images are allocated
 * apart from the workspace (the first call of each kind). */
int bayeslsh_reserve_workspace(blsh_ctx *ctx, size_t bytes, int32_t fixed);
int bayeslsh_workspace_bytes(blsh_ctx *ctx, size_t *bytes_host);

/* Wait for `stream`, then return (and clear) the first error a kernel of this
 * context raised since the last sync: BLSH_ETRUNCATED, BLSH_EBADID, BLSH_EINVAL
 * (empty set in bayeslsh_minhash_sigs), or BLSH_OK. */
int bayeslsh_sync(blsh_ctx *ctx, void *stream);

/* Thread-local description of the last failure of any call on this thread. */
const char *bayeslsh_last_error(void);
int bayeslsh_version(void);

/* Kernel timing: when enabled, every kernel launch of the context is bracketed
 * by HIP events on its stream.  bayeslsh_profile_read waits for the recorded
 * events and returns, for kernels whose name contains `name_substr`, the total
 * elapsed milliseconds and the number of launches since the last reset. */
int bayeslsh_profile_enable(blsh_ctx *ctx, int enable);
int bayeslsh_profile_reset(blsh_ctx *ctx);
int bayeslsh_profile_read(blsh_ctx *ctx, const char *name_substr, double *total_ms_host, int64_t *launches_host);

/* Launch tuning of a context (callers that want a fixed configuration, and
 * the autotuner).  Zero fields mean "library default".  The output is the same
 * whatever the tuning, except through k (which bayeslsh_verify_batched may
 * choose when called with a k of 0).
 *   gather: 1 = each lane gathers both signatures of its candidates directly
 *           (the only SRP gather scheme; reserved for alternatives).
 *           SRP signatures in OBJECT_MAJOR layout with rows of a multiple of
 *           128 hashes, 16-byte aligned, are read 128 hashes at a time (one
 *           16-byte gather per side serves the first 128/k levels), the fastest
 *           layout when most pairs end within the first 128 hashes.
 *   batch_inreg: batched calls run this many levels in registers before the
 *           undecided candidates are compacted into a survivor queue.
 *   batch_blocks_per_cu: blocks per CU of the batched tile kernel (4 waves
 *           each; every wave runs a contiguous range of tiles).
 *   batch_srp_tile: consecutive candidates of one cosine list per wave tile of
 *           the batched tile kernel: 128, 256 or 512 (2, 4 or 8 per lane).
 *   batch_mh_tile: the same for Jaccard lists: 64 or 128 (1 or 2 per lane).
 *           Both shapes are otherwise chosen by the autotuner (when the call
 *           autotunes k) or default to 256 and 64.
 *   tiles_accept_bitmask: 1 = the BLSH_TILES kernel tests acceptance with
 *           the per-level accept bitmask even when every level's accept set
 *           is an interval [min accept, n] (which it then tests with two
 *           bounds); the same output, for checking the bitmask path.
 *   batch_spill_cap: entries of each measure's survivor queue, split evenly
 *           into one region per wave of the tile kernel; a survivor that finds
 *           its wave's region full keeps running in registers (same result).
 *   acc_stage_cap: entries of the accepted-pair staging (single-call paths:
 *           verify, Lite, exhaustive; batched calls: at most 2^20).  Accepted
 *           pairs are first
 *           gathered into 256 slices with counters on separate cache lines
 *           (one counter serialises every wave's atomic) and appended to the
 *           caller's list after each launch; a pair that finds its slice full
 *           goes to the list directly (same output, slower).
 *   last_batch_*: set by the library after each batched call (the autotuned
 *           or given k of each measure, tile shapes, in-register levels and
 *           blocks per CU); ignored by bayeslsh_set_tuning.
 *   tiles_per_launch: BLSH_TILES calls run as launches of at most this many
 *           tiles (0 = 2^22; 1 .. 2^22), each followed by the copy of its
 *           staged accepted pairs to the caller's list; same output. */
typedef struct {
  int32_t gather;
  int32_t batch_inreg;
  int32_t batch_blocks_per_cu;
  int32_t last_batch_k_jaccard;
  int32_t last_batch_inreg;
  int32_t last_batch_blocks_per_cu;
  int32_t batch_spill_cap;   /* batched: survivor-queue entries per measure (0 = min(n_cand, 2^24)) */
  int32_t last_batch_k_cosine;
  int32_t acc_stage_cap;     /* accepted-pair staging entries (0 = 2^24 single-call, 2^20 batched) */
  int32_t batch_srp_tile;    /* 0, 128, 256 or 512 */
  int32_t batch_mh_tile;     /* 0, 64 or 128 */
  int32_t last_batch_srp_tile;
  int32_t last_batch_mh_tile;
  int32_t tiles_accept_bitmask;   /* 0 or 1 */
  int32_t tiles_per_launch;       /* 0 = 2^22 */
} blsh_tuning;
int bayeslsh_set_tuning(blsh_ctx *ctx, const blsh_tuning *tuning_host);
int bayeslsh_get_tuning(blsh_ctx *ctx, blsh_tuning *tuning_host);

/* ---------------- posterior tables (host, FP64) ---------------- */

/* Build (or fetch from the context's cache) the decision table of one
 * parameter set and copy it out.  For each level j (n = (j+1) k, j < n_levels):
 *   min_matches_host[j]  smallest m with Pr[S >= t | M(m,n)] >= epsilon, or n+1
 *                        (minMatches of Section 4.3)
 *   accept_host[j*words + w], words = (k*n_levels + 1 + 31)/32: bit m%32 of word
 *                        m/32 set iff m >= min_matches[j] and
 *                        Pr[|S - S_hat| < delta | M(m,n)] >= 1 - gamma
 *                        (the cache of concentration results of Section 4.3)
 * Jaccard probabilities use the Beta-binomial closed form (integer alpha,
 * beta) or the continued fraction of the regularized incomplete beta (other
 * alpha, beta); cosine ones use Gauss-Legendre quadrature over the angle theta with
 * r = 1 - theta/pi.  lite != 0 skips the concentration bits.  Either output
 * pointer may be NULL.  min_margin_host (optional) receives the smallest
 * distance of an evaluated probability from its threshold.  Host-only: ctx may
 * be NULL (no GPU needed; the table is then built without caching).
 * Near ties are refused: when some evaluated probability lies within 1e-9 of
 * its threshold (epsilon, or 1 - gamma), the decision at that (n, m) is not
 * fixed by FP64 evaluation, and the call returns BLSH_EINVAL with a message
 * naming the test and (n, m).  Every verification entry point (Algorithm 1,
 * Lite, exhaustive, batched, serving) builds its table through the same code
 * and refuses such a parameter set the same way, before enqueuing anything. */
int bayeslsh_posterior_table(blsh_ctx *ctx, blsh_measure measure, double t, double epsilon, double delta,
                             double gamma, blsh_prior prior, int32_t k, int32_t n_levels, int32_t lite,
                             int32_t *min_matches_host, uint32_t *accept_host, double *min_margin_host);

/* ---------------- signature generation (Section 4) ---------------- */

/* Minhash (Section 4.1): sigs[i][h] = min over e in set i of (a[h] e + b[h]) mod (2^31 - 1).
 * sets: kind BLSH_SETS (indices sorted or not); a[h] in [1, 2^31-1), b[h] in
 * [0, 2^31-1) (device arrays of n_hashes).  Output object-major uint32
 * [n_obj][n_hashes].  An empty set gets 0xFFFFFFFF everywhere and makes the
 * next bayeslsh_sync return BLSH_EINVAL. */
int bayeslsh_minhash_sigs(blsh_ctx *ctx, const blsh_vectors *sets, const uint32_t *a, const uint32_t *b,
                          int32_t n_hashes, uint32_t *sigs_out, void *stream);

/* Flags of bayeslsh_srp_sigs. */
enum {
  /* Cheaper storage of hash functions (Section 4.3): every generated plane
   * entry g (CSR vectors) is kept as the 2-byte code
   * c = floor((g + 8) * 2^16 / 16), clamped to [0, 65535], and used as the
   * middle of its cell, (c + 0.5) * 16 / 2^16 - 8, so |used - g| <= 2^-13
   * (about 1.22e-4; the paper prints 1e-4 for this encoding, which its cell
   * width of 2.44e-4 does not allow).  A generated entry never leaves
   * (-6.8, 6.8), so no entry saturates.  The plane table, when one is built,
   * holds the codes: 2 bytes per entry instead of 4.  The signature bits can
   * differ from the unflagged ones only where |r . x| <= 2^-13 sum |x_i|. */
  BLSH_SRP_PLANES_Q16 = 1
};

/* Sign random projections (Section 4.2): bit h of object i is 1 iff r_h . x_i >= 0,
 * packed LSB-first (hash h -> word h/32, bit h%32) in `layout`.
 *   DENSE vectors: planes = float R[dim][n_bits] (device); projections by an
 *     FP32 MFMA product.
 *   CSR vectors: planes = NULL; plane entries are generated on the fly:
 *     g(term, h) = float(z), z from Box-Muller in FP64 on the Philox-4x32-10
 *     words of counter (term, h/4, 0, 0) and key (seed lo32, seed hi32),
 *     u_i = (w_i + 0.5)/2^32, (z0,z1) = BoxMuller(u0,u1), (z2,z3) = BoxMuller(u2,u3),
 *     entry = z_{h mod 4}; projections accumulated in FP64.  The call reads
 *     the nonzero count (offsets[n_obj]) back, waiting for `stream`; when it
 *     exceeds 2 * dim and dim * n_bits * 4 bytes (2 with BLSH_SRP_PLANES_Q16)
 *     fit in 16 GiB, the entries of every term < dim are drawn once into a
 *     table in the context workspace and read from there (the same values;
 *     an index >= dim, outside the CSR contract, is drawn as it occurs rather
 *     than read past the table).
 * flags: 0 or BLSH_SRP_PLANES_Q16 (CSR only; with DENSE vectors it is
 * BLSH_EINVAL).  n_bits must be a multiple of 32 (DENSE: of 64). */
int bayeslsh_srp_sigs(blsh_ctx *ctx, const blsh_vectors *vecs, const float *planes, int32_t n_bits,
                      uint64_t seed, blsh_layout layout, int32_t flags, uint32_t *bits_out, void *stream);

/* ---------------- verification ---------------- */

/* Algorithm 1 (BayesLSH).  For each candidate: compare k hashes at a time;
 * prune when Pr[S >= t | M(m,n)] < epsilon; otherwise stop as soon as
 * Pr[|S - S_hat| < delta | M(m,n)] >= 1 - gamma and emit S_hat; a candidate
 * still undecided at n = n_max is emitted with its S_hat (ACCEPT_NMAX).
 * S_hat: Jaccard (m+alpha-1)/(n+alpha+beta-2) clamped to [0,1]; cosine
 * cos(pi (1 - max(0.5, m/n))).  Constraints: 0 < t, epsilon, delta, gamma < 1;
 * k in {16, 32, 64}; n_max % k == 0; n_max/k <= 64.  SRP signatures may be
 * OBJECT_MAJOR or WORD_MAJOR (WORD_MAJOR is the fast layout); minhash
 * signatures must be OBJECT_MAJOR with n_hashes % 4 == 0.
 * BLSH_TILES candidates (SRP; also bayeslsh_lite_verify, with h a multiple of
 * 128; the comparators and the allocation-free entry point refuse them with
 * BLSH_EINVAL): OBJECT_MAJOR rows, 16-byte aligned, of a multiple of 128
 * hashes, n_max a multiple of 128 up to 2048; tiles may come in any order of
 * their numbering.  Lite over tiles stages every position of a launch's tiles
 * for the exact similarity: 20 bytes of workspace per tile position (5 KiB
 * per tile), at most 2.7 GB (longer calls run as several launches).  A wave takes a
 * tile: it stages the first n_max hashes of its 32 members in LDS (one load
 * per 128-byte line), decides level 0 for the tile's pairs and finishes the
 * pairs level 0 does not prune from those rows.  Malformed tiles are reported
 * at the next bayeslsh_sync: a tile whose candidate numbers run outside
 * [0, n_cand) is skipped (nothing of it written), and positions past the
 * tile's n_rows / n_cols get code 0xFF (BLSH_EINVAL); a member id >= n_obj
 * gives its pairs code 0xFF (BLSH_EBADID). */
int bayeslsh_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs, double t,
                    double epsilon, double delta, double gamma, blsh_prior prior, int32_t k,
                    blsh_result *res, void *stream);

/* Algorithm 1 as bayeslsh_verify (same arguments, constraints and output),
 * for callers that cannot allocate device memory while they call: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The call allocates nothing (no hipMalloc or hipFree, no allocating library
 * routine): every buffer beyond the caller's inputs and outputs -- the slice
 * counters, the decision-table image, the survivor queue and the accepted-pair
 * staging -- lives in a fixed device array of the library, 16.7 MiB, one per
 * GPU (held until the process ends), sized for one launch of 2^20 candidates;
 * a longer call runs as several launches, so no input size exceeds it.  The
 * array keeps the last call's contents; a call clears what it relies on, on
 * `stream`, before its first launch.  Calls that overlap on one GPU -- from
 * any context or stream -- share the array and race: the caller serialises
 * them.  A parameter set seen for the first time has its table built on the
 * host (host memory only) and its image copied into the array on `stream`.
 * Candidate kinds: PAIRS, QUERY_LISTS and ALL_PAIRS; BLSH_TILES is refused
 * (BLSH_EINVAL: its per-wave staging is sized by the call).
 * Errors: as bayeslsh_verify; BLSH_EINVAL for a context on a device numbered
 * 64 or above (no scratch array is kept there). */
int bayeslsh_verify_noalloc(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs, double t,
                            double epsilon, double delta, double gamma, blsh_prior prior, int32_t k,
                            blsh_result *res, void *stream);

/* Algorithm 2 (BayesLSH-Lite).  Prune as above using at most h hashes
 * (h % k == 0, h <= n_max); survivors get their exact similarity from `exact`
 * (cosine: DENSE or CSR, sums in FP64; Jaccard: SETS) and are emitted iff
 * s > t, with s as acc_val.  Survivor codes are LITE_EXACT at level h/k - 1. */
int bayeslsh_lite_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs,
                         const blsh_vectors *exact, double t, double epsilon, blsh_prior prior, int32_t h,
                         int32_t k, blsh_result *res, void *stream);

/* Exact similarity of every candidate (the quantity Algorithm 2 computes for
 * its survivors): Jaccard |A n B| / |A u B| of SETS vectors, cosine of DENSE
 * or CSR vectors with sums in FP64.  sim_out: device double[n_cand], one value
 * per candidate index; a candidate with an id >= n_obj gets NaN and makes the
 * next bayeslsh_sync return BLSH_EBADID.  Used to draw the similarity sample
 * that bayeslsh_fit_prior turns into a prior. */
int bayeslsh_exact_similarity(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_vectors *vecs,
                              double *sim_out, void *stream);

/* LSH banding candidate generation (Section 2): the first n_bands * band_bits
 * bits of each object's sign-random-projection signature (`band_sigs`, an
 * SRP set drawn independently of the verification bits; either layout) are
 * cut into n_bands band keys of band_bits bits; two objects whose keys are
 * equal in some band form a candidate pair, emitted once, in the first band
 * where they collide.  max_bucket > 0 keeps only the first max_bucket members
 * (by id) of each bucket.  Output order: band by band, buckets by increasing
 * key, then the pairs (x, y), x < y, of the bucket's members (by id):
 * order_tile = 0, row-major over member positions; order_tile = 16, by 16 x 16
 * tiles of member positions (tile rows, then tile columns, row-major inside a
 * tile), so that a run of 256 candidates touches about 32 objects -- the
 * order the verification kernels read best.  x_out, y_out:
 * device uint32[capacity].  *n_pairs_host receives the number of pairs; the
 * call waits for `stream`.  More pairs than capacity: the first `capacity` are
 * written and BLSH_ETRUNCATED is returned; order_tile other than 0 or 16
 * gives BLSH_EINVAL.  Uses the context workspace (about 8 * n_obj * (n_bands
 * + 6) bytes) and, with tiles, a context buffer of 48 bytes per tile of the
 * largest band. */
int bayeslsh_band_candidates(blsh_ctx *ctx, const blsh_sigs *band_sigs, int32_t n_bands, int32_t band_bits,
                             int32_t max_bucket, int32_t order_tile, uint32_t *x_out, uint32_t *y_out,
                             int64_t capacity, int64_t *n_pairs_host, void *stream);

/* LSH banding (Section 2) as bucket tiles: the candidates of
 * bayeslsh_band_candidates with order_tile = 16 -- the same pairs with the same
 * candidate indices -- handed over as one blsh_tile per 16 x 16 tile of a
 * bucket's member pairs (the tile's 32 member ids, its keep mask and the index
 * of its first candidate) instead of one id pair per candidate: 192 bytes per
 * up to 256 candidates instead of 8 bytes per candidate.
 *   tiles_out    device blsh_tile[tiles_capacity], 16-byte aligned: band by
 *                band, buckets by increasing key, tile rows then tile columns;
 *   *n_tiles_host, *n_pairs_host  tiles and candidates; the call waits for
 *                `stream`.  More tiles than the capacity: the first
 *                tiles_capacity are written, BLSH_ETRUNCATED.
 * Pass the outputs as a BLSH_TILES candidate set (tiles, n_tiles, n_cand =
 * *n_pairs_host). */
int bayeslsh_band_tiles(blsh_ctx *ctx, const blsh_sigs *band_sigs, int32_t n_bands, int32_t band_bits,
                        int32_t max_bucket, blsh_tile *tiles_out, int64_t tiles_capacity, int64_t *n_tiles_host,
                        int64_t *n_pairs_host, void *stream);

/* Learned Jaccard prior (Section 4.1): Beta(alpha, beta) fitted to a random
 * sample of candidate-pair similarities s_1..s_r (host array) by the method
 * of moments: with the sample mean m and variance v = sum (s_i - m)^2 / r,
 *   alpha = m (m (1 - m) / v - 1),  beta = (1 - m) (m (1 - m) / v - 1).
 * When no Beta has these moments (r < 2, v = 0 or v >= m (1 - m)) or the fit
 * exceeds 1e6, the uniform prior {1, 1} is written and *uniform_host (may be
 * NULL) is set to 1.  Host-only; BLSH_EINVAL if a value is outside [0, 1]. */
int bayeslsh_fit_prior(const double *sim_host, int64_t r, blsh_prior *prior_out, int32_t *uniform_host);

/* Exhaustive comparator: every candidate compares all n_max hashes (no early
 * exit, object-major rows read whole), then
 *   mode REPLAY:      the decision sequence of Algorithm 1 is replayed on the
 *                     per-level counts -> output identical to bayeslsh_verify;
 *   mode REPLAY_LITE: the same for Algorithm 2 with budget h, then exact
 *                     similarity on survivors -> identical to bayeslsh_lite_verify;
 *   mode MLE:         the classical estimate m/n_max (cosine: r2c(m/n_max)),
 *                     emitted iff >= t (Section 3; "LSH Approx" of Section 5.1);
 *                     codes are ACCEPT_NMAX / PRUNED at level n_max/k - 1.
 * `exact` and h are used by REPLAY_LITE only. */
typedef enum { BLSH_REPLAY = 0, BLSH_REPLAY_LITE = 1, BLSH_MLE = 2 } blsh_exhaustive_mode;
int bayeslsh_exhaustive_verify(blsh_ctx *ctx, const blsh_candidates *cand, const blsh_sigs *sigs,
                               const blsh_vectors *exact, double t, double epsilon, double delta,
                               double gamma, blsh_prior prior, int32_t k, int32_t h,
                               blsh_exhaustive_mode mode, blsh_result *res, void *stream);

/* Batched verification (Algorithm 1) of many query lists in one call: list i
 * verifies the candidates cand[offset .. offset+length) against its query
 * object, under its own measure and threshold t, with shared epsilon, delta,
 * gamma and Jaccard prior.  Lists use `jaccard_sigs` (minhash,
 * OBJECT_MAJOR) or `cosine_sigs` (SRP, either layout; OBJECT_MAJOR rows of a
 * multiple of 128 hashes, 16-byte aligned, are read 128 hashes per gather);
 * a set a batch does not use may be NULL.  Candidate index = position in
 * cand, as for QUERY_LISTS; positions no list covers are left untouched.  At
 * most 32 distinct thresholds per call.
 * Execution: one graph of kernels on a fixed grid (every wave runs a
 * contiguous range of tiles; candidates undecided after `batch_inreg` levels
 * are compacted into a survivor queue, which a second kernel drains).
 * k_jaccard and k_cosine (16, 32 or 64) fix each measure's chunk size; 0 lets
 * an autotuner pick it, and then also the in-register levels and the grid,
 * by timing this batch shape (cached per context).  The k used are written to
 * k_used_host[0] (Jaccard) and k_used_host[1] (cosine); k_used_host may be
 * NULL.  k changes the check points of the algorithm and hence the output.
 * Consecutive batched calls on one context must use the same stream (or be
 * synchronised): they share the context's device-side batch descriptor. */
typedef struct {
  blsh_measure measure;
  double t;
  uint32_t query;
  int64_t offset;
  int64_t length;
} blsh_list_desc;
int bayeslsh_verify_batched(blsh_ctx *ctx, const blsh_list_desc *lists_host, int64_t n_lists, const uint32_t *cand,
                            int64_t n_cand, const blsh_sigs *jaccard_sigs, const blsh_sigs *cosine_sigs,
                            double epsilon, double delta, double gamma, blsh_prior jaccard_prior, int32_t k_jaccard,
                            int32_t k_cosine, int32_t *k_used_host, blsh_result *res, void *stream);

/* Exhaustive comparator for a batch: the same lists, but every candidate
 * compares all n_max hashes of its object-major row with the query's, and
 * the decision sequence of Algorithm 1 is replayed on the per-level counts,
 * so the output equals bayeslsh_verify_batched's at the same k pair (both
 * required for the measures the batch uses).
 * Signatures must be OBJECT_MAJOR with 16-byte aligned rows; SRP n_max one of
 * 128, 256, 512, 1024, 2048; minhash n_max a multiple of 64. */
int bayeslsh_exhaustive_batched(blsh_ctx *ctx, const blsh_list_desc *lists_host, int64_t n_lists, const uint32_t *cand,
                                int64_t n_cand, const blsh_sigs *jaccard_sigs, const blsh_sigs *cosine_sigs,
                                double epsilon, double delta, double gamma, blsh_prior jaccard_prior,
                                int32_t k_jaccard, int32_t k_cosine, blsh_result *res, void *stream);

/* ---------------- serving ---------------- */

/* A serving loop answers similarity queries against a resident signature
 * index: each request is a query object, its candidate ids (host memory) and a
 * threshold t, verified with Algorithm 1 (epsilon, delta, gamma and k fixed at
 * creation).  A scheduler thread (owned by the server) admits requests FIFO
 * as long as an in-flight slot is free and their candidate ids fit in a device
 * arena of mem_budget_bytes (4 bytes per candidate), then runs continuous
 * batching: each device iteration verifies the next chunk of every admitted
 * request (fair shares of max_batch_candidates) in one batched launch, so
 * requests that arrive while others run join the next iteration.  A request
 * completes when its last chunk's accepted pairs have been copied back; its
 * output does not depend on the requests it was batched with.
 * The server uses `ctx` exclusively until bayeslsh_server_destroy; the index
 * signatures must stay valid meanwhile. */
typedef struct {
  size_t mem_budget_bytes;       /* device arena for candidate ids (admission limit) */
  int32_t max_active;            /* requests admitted at once */
  int32_t k;                     /* 16, 32 or 64 */
  int64_t max_batch_candidates;  /* candidates per device iteration */
  double epsilon, delta, gamma;
  blsh_prior prior;              /* Jaccard prior (cosine: {1,1}) */
} blsh_server_config;

/* Result of a finished request.  The arrays are owned by the server and stay
 * valid until bayeslsh_server_release.  acc_idx are positions in the
 * request's candidate list, in increasing order.  Times are seconds on the
 * server's clock (bayeslsh_server_clock). */
typedef struct {
  int64_t n_candidates;
  int64_t n_accepted;
  const uint64_t *acc_idx_host;
  const float *acc_val_host;
  double submit_time_s, admit_time_s, done_time_s;
  int32_t status;
} blsh_request_result;

typedef struct blsh_server blsh_server;
int bayeslsh_server_create(blsh_ctx *ctx, const blsh_sigs *index, const blsh_server_config *cfg, blsh_server **out);
/* Copies the candidate ids; rejects ids >= n_obj (BLSH_EINVAL) and requests larger
 * than the arena (BLSH_ENOMEM). */
int bayeslsh_server_submit(blsh_server *srv, uint32_t query, const uint32_t *cand_host, int64_t n_cand, double t,
                           int64_t *request_id);
/* As bayeslsh_server_submit for candidate ids already in device memory (for
 * instance from bayeslsh_band_candidates): nothing is copied on the host; the
 * server copies them device to device into its arena when it admits the
 * request, on its own stream, which does not wait for the caller's streams:
 * the ids must be written (synchronised) before the call, and cand_dev must
 * stay valid and unchanged until the request is finished (poll/wait report
 * it).  Ids are checked on the device only: a
 * candidate with an id >= n_obj is never accepted, the other candidates are
 * verified as usual, and the request finishes with status BLSH_EBADID (its
 * accepted list still holds the valid candidates' results).  A query id >=
 * n_obj is rejected here (BLSH_EINVAL), and so is a cand_dev that is not
 * device memory of the server's GPU holding n_cand ids (host, managed or
 * another GPU's memory, or a range past the end of its allocation); requests
 * larger than the arena: BLSH_ENOMEM.  Any pending status of `ctx` is cleared
 * when the server is created. */
int bayeslsh_server_submit_device(blsh_server *srv, uint32_t query, const uint32_t *cand_dev, int64_t n_cand,
                                  double t, int64_t *request_id);
/* BLSH_OK (finished; *out filled), BLSH_EAGAIN (pending) or an error. */
int bayeslsh_server_poll(blsh_server *srv, int64_t request_id, blsh_request_result *out);
int bayeslsh_server_wait(blsh_server *srv, int64_t request_id, blsh_request_result *out);
int bayeslsh_server_release(blsh_server *srv, int64_t request_id);
/* Device iterations run, requests waiting and admitted now, and admission rounds
 * that had to leave requests waiting for a slot or arena space.  Any pointer may be NULL. */
int bayeslsh_server_stats(blsh_server *srv, int64_t *iterations_host, int64_t *pending_host, int64_t *active_host,
                          int64_t *deferred_host);
double bayeslsh_server_clock(blsh_server *srv);
void bayeslsh_server_destroy(blsh_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* BAYESLSH_H */
