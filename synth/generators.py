"""Seeded workload generators (numpy only).

Every generator is a pure function of its arguments and seed.  Shapes and
distributions follow the benchmark workloads, which stand in for the paper's
datasets (Section 5, Table 1): binary sets
for Jaccard similarity, sparse tf-idf vectors and dense embeddings for
cosine similarity, and LSH-banded candidate pairs (Section 2, candidate
generation).  The random draws a hash family needs (minhash coefficients,
dense Gaussian planes) are produced here and handed to both the GPU path
and the oracle as inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SEED_BASE", "MINHASH_PRIME", "SetCollection", "SparseCorpus", "DenseMixture",
    "jaccard_sets", "minhash_coeffs", "gaussian_planes", "dense_mixture",
    "tfidf_corpus", "band_candidates", "random_pairs", "all_pairs_count",
    "query_lists", "calibration_minhash", "calibration_bits", "pack_bits",
    "subsample_pairs",
]

SEED_BASE = 11101328
# Range of the universal-hash coefficients drawn for the minhash family:
# a in [1, P), b in [0, P) with P the Mersenne prime 2^31 - 1.
MINHASH_PRIME = (1 << 31) - 1


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# Sets (Jaccard workloads)
# ----------------------------------------------------------------------------
@dataclass
class SetCollection:
    offsets: np.ndarray          # int64 [n+1]
    elems: np.ndarray            # uint32, sorted and unique within each set
    group: np.ndarray            # int32 [n]: planted group id, -1 for background sets
    is_base: np.ndarray          # bool  [n]: the unmodified base of a planted group
    vocab: int

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def row(self, i: int) -> np.ndarray:
        return self.elems[self.offsets[i]:self.offsets[i + 1]]


def _csr_from_rows(rows):
    lens = np.fromiter((len(r) for r in rows), dtype=np.int64, count=len(rows))
    offsets = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    elems = np.concatenate(rows).astype(np.uint32) if rows else np.zeros(0, np.uint32)
    return offsets, elems


def jaccard_sets(n_sets=2000, vocab=100_000, median=60.0, sigma=0.8, n_groups=100,
                 group_size=5, frac_lo=0.1, frac_hi=0.4, seed=SEED_BASE + 1) -> SetCollection:
    """Binary sets with lognormal sizes and planted near-duplicate groups.

    Each planted group is a base set plus ``group_size - 1`` members; a member
    replaces a fraction f ~ U(frac_lo, frac_hi) of the base's elements with
    ids that are not in the base.  Background sets draw their elements
    uniformly without replacement.  Group sets sit at random positions.
    """
    rng = _rng(seed)
    n_planted = n_groups * group_size
    assert n_planted <= n_sets
    sizes = np.maximum(1, np.rint(np.exp(math.log(median) + sigma * rng.standard_normal(n_sets)))).astype(np.int64)
    sizes = np.minimum(sizes, vocab // 2)
    pos = rng.permutation(n_sets)
    rows = [None] * n_sets
    group = np.full(n_sets, -1, np.int32)
    is_base = np.zeros(n_sets, bool)
    slot = 0
    for g in range(n_groups):
        base_pos = pos[slot]
        base = np.sort(rng.choice(vocab, size=sizes[base_pos], replace=False))
        rows[base_pos] = base
        group[base_pos] = g
        is_base[base_pos] = True
        slot += 1
        for _ in range(group_size - 1):
            p = pos[slot]
            slot += 1
            f = rng.uniform(frac_lo, frac_hi)
            n_rep = int(round(f * len(base)))
            keep = rng.choice(len(base), size=len(base) - n_rep, replace=False)
            fresh = []
            base_set = set(base.tolist())
            while len(fresh) < n_rep:
                cand = rng.integers(0, vocab, size=2 * (n_rep - len(fresh)) + 4)
                for c in cand.tolist():
                    if c not in base_set and c not in fresh:
                        fresh.append(c)
                        if len(fresh) == n_rep:
                            break
            rows[p] = np.sort(np.concatenate([base[keep], np.asarray(fresh, dtype=np.int64)]))
            group[p] = g
    for p in pos[slot:]:
        rows[p] = np.sort(rng.choice(vocab, size=sizes[p], replace=False))
    offsets, elems = _csr_from_rows(rows)
    return SetCollection(offsets, elems, group, is_base, vocab)


def minhash_coeffs(n_hashes: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Coefficients (a_i, b_i) of n universal hash functions e -> (a_i e + b_i) mod P."""
    rng = _rng(seed)
    a = rng.integers(1, MINHASH_PRIME, size=n_hashes, dtype=np.int64).astype(np.uint32)
    b = rng.integers(0, MINHASH_PRIME, size=n_hashes, dtype=np.int64).astype(np.uint32)
    return a, b


# ----------------------------------------------------------------------------
# Dense embeddings (cosine workloads)
# ----------------------------------------------------------------------------
@dataclass
class DenseMixture:
    x: np.ndarray        # float32 [n, d], unit norm (normalized in float64)
    comp: np.ndarray     # int32 [n]
    mu: np.ndarray       # float64 [n_comp, d]
    sigma: np.ndarray    # float64 [n_comp]


def gaussian_planes(d: int, n_bits: int, seed: int) -> np.ndarray:
    """Standard-normal plane matrix R, float32 [d, n_bits] (column b is plane b)."""
    rng = _rng(seed)
    return rng.standard_normal((d, n_bits)).astype(np.float32)


def dense_mixture(n=1_000_000, d=256, n_comp=1000, sig_lo=0.02, sig_hi=0.06,
                  seed=SEED_BASE + 4, chunk=1 << 17) -> DenseMixture:
    """Unit vectors from a Gaussian mixture: x = normalize(mu_c + sigma_c z)."""
    rng = _rng(seed)
    mu = rng.standard_normal((n_comp, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    sig = rng.uniform(sig_lo, sig_hi, size=n_comp)
    comp = rng.integers(0, n_comp, size=n).astype(np.int32)
    x = np.empty((n, d), np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        c = comp[s:e]
        v = mu[c] + sig[c, None] * rng.standard_normal((e - s, d))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        x[s:e] = v.astype(np.float32)
    return DenseMixture(x, comp, mu, sig)


# ----------------------------------------------------------------------------
# Sparse tf-idf corpus (cosine, Lite workload)
# ----------------------------------------------------------------------------
@dataclass
class SparseCorpus:
    offsets: np.ndarray      # int64 [n+1]
    indices: np.ndarray      # uint32, sorted ascending and unique within a row
    values: np.ndarray       # float32, each row L2-normalized in float64 then rounded
    dim: int
    dup_source: np.ndarray = field(default=None)  # int64 [n]: source doc of a planted duplicate, -1 otherwise

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def row(self, i: int):
        s, e = self.offsets[i], self.offsets[i + 1]
        return self.indices[s:e], self.values[s:e]


def tfidf_corpus(n_docs=100_000, dim=1 << 20, mean_nnz=100, zipf_s=1.1, dup_frac=0.05,
                 rep_lo=0.1, rep_hi=0.3, jit_lo=0.8, jit_hi=1.2, seed=SEED_BASE + 2) -> SparseCorpus:
    """tf-idf vectors: Poisson(mean_nnz) distinct terms per row, truncated-Zipf term
    ranks mapped through a seeded permutation of [0, dim), tf = multiplicity,
    idf = ln(N / df).

    A fraction ``dup_frac`` of the documents are planted near-duplicates: a copy of
    a random source document with 10-30% of its distinct terms replaced by fresh
    Zipf draws and every weight multiplied by U(0.8, 1.2).  Terms present in
    every document get idf 0 and are dropped; a row left empty gets one private
    term of weight 1 (never observed at the default sizes).
    """
    rng = _rng(seed)
    ranks = np.arange(1, dim + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-zipf_s))
    cdf /= cdf[-1]
    rank2term = rng.permutation(dim).astype(np.int64)

    def draw(k):
        r = np.searchsorted(cdf, rng.random(k), side="right")
        return rank2term[np.minimum(r, dim - 1)]

    n_dup = int(round(dup_frac * n_docs))
    n_base = n_docs - n_dup
    nnz = np.maximum(1, rng.poisson(mean_nnz, size=n_base)).astype(np.int64)
    # Each document draws Zipf tokens until it holds nnz distinct terms; tf is the
    # multiplicity of a term among the tokens drawn up to that point.
    b_term_rows, tf_rows = [], []
    for d in range(n_base):
        want = int(nnz[d])
        tok = draw(3 * want + 32)
        u, first, inv = np.unique(tok, return_index=True, return_inverse=True)
        if len(u) > want:
            cut = np.sort(first)[want - 1] + 1
            u, inv = np.unique(tok[:cut], return_inverse=True)
        cnt = np.bincount(inv, minlength=len(u))
        b_term_rows.append(u)
        tf_rows.append(cnt)
    b_term = np.concatenate(b_term_rows)
    tf = np.concatenate(tf_rows).astype(np.int64)
    b_off = np.zeros(n_base + 1, np.int64)
    np.cumsum([len(r) for r in b_term_rows], out=b_off[1:])

    # planted duplicates (raw term/tf rows)
    src = rng.integers(0, n_base, size=n_dup)
    d_terms, d_tf, d_jit = [], [], []
    for s in src.tolist():
        t = b_term[b_off[s]:b_off[s + 1]]
        c = tf[b_off[s]:b_off[s + 1]]
        f = rng.uniform(rep_lo, rep_hi)
        n_rep = int(round(f * len(t)))
        keep = np.sort(rng.choice(len(t), size=len(t) - n_rep, replace=False))
        nt = np.concatenate([t[keep], draw(n_rep)])
        nc = np.concatenate([c[keep], np.ones(n_rep, np.int64)])
        u, inv = np.unique(nt, return_inverse=True)
        uc = np.bincount(inv, weights=nc).astype(np.int64)
        d_terms.append(u)
        d_tf.append(uc)
        d_jit.append(rng.uniform(jit_lo, jit_hi, size=len(u)))

    all_terms = np.concatenate([b_term] + d_terms)
    all_tf = np.concatenate([tf] + d_tf).astype(np.float64)
    row_len = np.concatenate([np.diff(b_off), np.array([len(u) for u in d_terms], np.int64)])
    jit = np.concatenate([np.ones(len(b_term))] + d_jit)
    df = np.bincount(all_terms, minlength=dim)
    idf = np.log(n_docs / np.maximum(df, 1))
    w = all_tf * idf[all_terms] * jit

    # place documents at random positions
    order = rng.permutation(n_docs)          # order[new_pos] = old doc id
    old_off = np.zeros(n_docs + 1, np.int64)
    np.cumsum(row_len, out=old_off[1:])
    rows_i, rows_v = [], []
    dup_source = np.full(n_docs, -1, np.int64)
    new_of_old = np.empty(n_docs, np.int64)
    new_of_old[order] = np.arange(n_docs)
    spare = dim  # private terms for empty rows are taken from the top of the id space
    for new in range(n_docs):
        old = order[new]
        s, e = old_off[old], old_off[old + 1]
        ti, tv = all_terms[s:e], w[s:e]
        keep = tv > 0
        ti, tv = ti[keep], tv[keep]
        if len(ti) == 0:
            spare -= 1
            ti, tv = np.array([spare], np.int64), np.array([1.0])
        tv = tv / np.sqrt(np.sum(tv * tv))
        rows_i.append(ti)
        rows_v.append(tv.astype(np.float32))
        if old >= n_base:
            dup_source[new] = new_of_old[src[old - n_base]]
    offsets, _ = _csr_from_rows(rows_i)
    indices = np.concatenate(rows_i).astype(np.uint32)
    values = np.concatenate(rows_v).astype(np.float32)
    return SparseCorpus(offsets, indices, values, dim, dup_source)


def _sparse_project(corpus: SparseCorpus, n_planes: int, seed: int) -> np.ndarray:
    """Projections of every row onto fresh Gaussian planes (float64), used only to
    band candidates; this draw is independent of any verification signature."""
    import scipy.sparse as sp
    rng = _rng(seed)
    used, inv = np.unique(corpus.indices, return_inverse=True)
    g = rng.standard_normal((len(used), n_planes))
    x = sp.csr_matrix((corpus.values.astype(np.float64), inv.astype(np.int64), corpus.offsets),
                      shape=(corpus.n, len(used)))
    return np.asarray(x @ g)


def band_candidates(proj: np.ndarray, n_bands: int, band_bits: int, max_bucket: int | None = None):
    """LSH banding on sign bits of ``proj`` (float [n, n_bands*band_bits]).

    All pairs that share a band key become candidates, emitted bucket-major
    (band by band, bucket by bucket, members in id order, i < j); a pair that
    already collided in an earlier band is dropped (first-band dedupe).
    Returns (x, y) uint32 arrays.
    """
    n = proj.shape[0]
    bits = (proj >= 0)
    keys = np.zeros((n, n_bands), np.int64)
    for b in range(n_bands):
        blk = bits[:, b * band_bits:(b + 1) * band_bits].astype(np.int64)
        keys[:, b] = (blk << np.arange(band_bits, dtype=np.int64)).sum(1)
    tri_cache = {}
    xs, ys = [], []
    for b in range(n_bands):
        k = keys[:, b]
        order = np.lexsort((np.arange(n), k))
        ks = k[order]
        cut = np.flatnonzero(np.diff(ks)) + 1
        starts = np.concatenate([[0], cut])
        ends = np.concatenate([cut, [n]])
        bx, by = [], []
        for s, e in zip(starts.tolist(), ends.tolist()):
            sz = e - s
            if sz < 2:
                continue
            mem = order[s:e]
            if max_bucket is not None and sz > max_bucket:
                mem = mem[:max_bucket]
                sz = max_bucket
            if sz not in tri_cache:
                tri_cache[sz] = np.triu_indices(sz, 1)
            ii, jj = tri_cache[sz]
            bx.append(mem[ii])
            by.append(mem[jj])
        if not bx:
            continue
        bx = np.concatenate(bx)
        by = np.concatenate(by)
        if b > 0:
            keep = np.ones(len(bx), bool)
            step = 1 << 22
            for s in range(0, len(bx), step):
                e = min(len(bx), s + step)
                keep[s:e] = ~(keys[bx[s:e], :b] == keys[by[s:e], :b]).any(1)
            bx, by = bx[keep], by[keep]
        xs.append(bx.astype(np.uint32))
        ys.append(by.astype(np.uint32))
    if not xs:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    return np.concatenate(xs), np.concatenate(ys)


def sparse_band_candidates(corpus: SparseCorpus, n_bands=16, band_bits=10, seed=SEED_BASE + 102):
    return band_candidates(_sparse_project(corpus, n_bands * band_bits, seed), n_bands, band_bits)


def sparse_band_bits(corpus: SparseCorpus, n_bands=16, band_bits=10, seed=SEED_BASE + 102) -> np.ndarray:
    """The sign bits that sparse_band_candidates bands, packed 32 to a uint32
    word, least significant bit first: bit b * band_bits + t of an object is
    the sign of its projection on plane b * band_bits + t (the rest of the
    last word is zero).  Shape [n, ceil(n_bands * band_bits / 32)]."""
    nb = n_bands * band_bits
    proj = _sparse_project(corpus, nb, seed)
    w = (nb + 31) // 32
    bits = np.zeros((corpus.n, w * 32), np.uint64)
    bits[:, :nb] = proj >= 0
    return (bits.reshape(corpus.n, w, 32) << np.arange(32, dtype=np.uint64)).sum(2).astype(np.uint32)


def dense_band_candidates(x: np.ndarray, n_bands=16, band_bits=12, seed=SEED_BASE + 104, max_bucket=None):
    g = _rng(seed).standard_normal((x.shape[1], n_bands * band_bits))
    proj = x.astype(np.float64) @ g
    return band_candidates(proj, n_bands, band_bits, max_bucket)


__all__ += ["sparse_band_candidates", "sparse_band_bits", "dense_band_candidates"]


# ----------------------------------------------------------------------------
# Candidate helpers
# ----------------------------------------------------------------------------
def all_pairs_count(n: int) -> int:
    return n * (n - 1) // 2


def random_pairs(n_obj: int, n_pairs: int, seed: int):
    rng = _rng(seed)
    x = rng.integers(0, n_obj, size=n_pairs).astype(np.uint32)
    y = rng.integers(0, n_obj, size=n_pairs).astype(np.uint32)
    return x, y


def subsample_pairs(n_pairs: int, n_sample: int, seed: int) -> np.ndarray:
    """Sorted distinct indices into a candidate array (for sampled parity checks)."""
    rng = _rng(seed)
    n_sample = min(n_sample, n_pairs)
    return np.sort(rng.choice(n_pairs, size=n_sample, replace=False)).astype(np.int64)


def query_lists(n_lists: int, n_obj: int, len_lo_exp: float, len_hi_exp: float, members,
                member_frac=0.01, seed=SEED_BASE + 3, max_total=None):
    """Candidate lists of log-uniform length 10^U(lo, hi).

    ``members(q)`` returns the ids related to query q (its planted group or
    mixture component); ``member_frac`` of each list is drawn from them and the
    rest uniformly without replacement.  Each list is sorted.  Returns
    (query uint32 [L], offsets int64 [L+1], cand uint32 [total]).
    """
    rng = _rng(seed)
    lens = np.floor(10.0 ** rng.uniform(len_lo_exp, len_hi_exp, size=n_lists)).astype(np.int64)
    lens = np.minimum(lens, n_obj - 1)
    if max_total is not None and lens.sum() > max_total:
        lens = np.maximum(1, (lens * (max_total / lens.sum())).astype(np.int64))
    queries = rng.integers(0, n_obj, size=n_lists).astype(np.uint32)
    offsets = np.zeros(n_lists + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    cand = np.empty(int(offsets[-1]), np.uint32)
    for i in range(n_lists):
        L = int(lens[i])
        mem = np.asarray(members(int(queries[i])), dtype=np.int64)
        n_mem = min(len(mem), int(round(member_frac * L)))
        pick_m = rng.choice(mem, size=n_mem, replace=False) if n_mem else np.zeros(0, np.int64)
        need = L - n_mem
        if need > n_obj // 4:
            pool = rng.permutation(n_obj)[:need + n_mem + 1]
        else:
            pool = np.unique(rng.integers(0, n_obj, size=int(need * 1.1) + 16))
            while len(pool) < need + n_mem + 1:
                pool = np.unique(np.concatenate([pool, rng.integers(0, n_obj, size=need + 16)]))
            pool = rng.permutation(pool)
        pool = pool[~np.isin(pool, pick_m)][:need]
        c = np.sort(np.concatenate([pick_m, pool]))
        cand[offsets[i]:offsets[i] + len(c)] = c
        if len(c) < L:   # only if the member pool overlapped; pad with a repeat of the last id
            cand[offsets[i] + len(c):offsets[i + 1]] = c[-1]
    return queries, offsets, cand


# ----------------------------------------------------------------------------
# Calibration inputs: signatures whose hashes agree independently with prob S
# ----------------------------------------------------------------------------
def calibration_minhash(n_pairs: int, n_hashes: int, s: np.ndarray, seed: int):
    """Signature rows (2*n_pairs objects, uint32 [2n, n_hashes]) where object 2i+1
    agrees with object 2i on each hash independently with probability s[i]."""
    rng = _rng(seed)
    a = rng.integers(0, 1 << 31, size=(n_pairs, n_hashes), dtype=np.int64)
    other = rng.integers(0, (1 << 31) - 1, size=(n_pairs, n_hashes), dtype=np.int64)
    other = np.where(other >= a, other + 1, other)  # any value except a
    agree = rng.random((n_pairs, n_hashes)) < s[:, None]
    b = np.where(agree, a, other)
    sig = np.empty((2 * n_pairs, n_hashes), np.uint32)
    sig[0::2] = a
    sig[1::2] = b
    return sig


def calibration_bits(n_pairs: int, n_bits: int, r: np.ndarray, seed: int):
    """Bit signatures (0/1 uint8 [2n, n_bits]) agreeing per bit with probability r[i]."""
    rng = _rng(seed)
    a = rng.integers(0, 2, size=(n_pairs, n_bits), dtype=np.uint8)
    agree = rng.random((n_pairs, n_bits)) < r[:, None]
    b = np.where(agree, a, 1 - a).astype(np.uint8)
    bits = np.empty((2 * n_pairs, n_bits), np.uint8)
    bits[0::2] = a
    bits[1::2] = b
    return bits


def pack_bits(bits01: np.ndarray) -> np.ndarray:
    """Pack 0/1 bits [n, n_bits] into uint32 words [n, n_bits/32], bit i -> word i//32, bit i%32."""
    n, nb = bits01.shape
    assert nb % 32 == 0
    b = bits01.reshape(n, nb // 32, 32).astype(np.uint64)
    w = (b << np.arange(32, dtype=np.uint64)).sum(2)
    return w.astype(np.uint32)


# ----------------------------------------------------------------------------
# Large-scale variants (vectorised) for the batched and serving workloads
# ----------------------------------------------------------------------------
def jaccard_sets_large(n_sets=1_000_000, vocab=100_000, median=60.0, sigma=0.8, n_groups=50_000, group_size=5,
                       frac_lo=0.1, frac_hi=0.4, seed=SEED_BASE + 5) -> SetCollection:
    """The planted-group set collection at scale, drawn without per-set Python
    loops.  Elements are drawn with replacement and deduplicated (at these
    sizes a set loses an element with probability ~ size^2 / (2 vocab));
    a member keeps each base element with probability 1 - f and replaces the
    others by uniform ids (dropped if they collide with the base)."""
    rng = _rng(seed)
    sizes = np.maximum(1, np.rint(np.exp(math.log(median) + sigma * rng.standard_normal(n_sets)))).astype(np.int64)
    sizes = np.minimum(sizes, vocab // 2)
    pos = rng.permutation(n_sets)
    group = np.full(n_sets, -1, np.int32)
    is_base = np.zeros(n_sets, bool)
    n_planted = n_groups * group_size
    gpos = pos[:n_planted].reshape(n_groups, group_size)
    group[gpos.ravel()] = np.repeat(np.arange(n_groups, dtype=np.int32), group_size)
    is_base[gpos[:, 0]] = True
    # independent rows: background sets and group bases
    indep = np.concatenate([gpos[:, 0], pos[n_planted:]])
    lens = sizes[indep]
    owner = np.repeat(indep, lens)
    el = rng.integers(0, vocab, size=int(lens.sum()), dtype=np.int64)
    key = np.unique(owner.astype(np.int64) * vocab + el)
    # members derived from their base
    base_of = np.repeat(gpos[:, 0], group_size - 1)
    members = gpos[:, 1:].ravel()
    f = rng.uniform(frac_lo, frac_hi, size=len(members))
    b_owner = key // vocab
    b_elem = key - b_owner * vocab
    b_start = np.searchsorted(b_owner, base_of, side="left")
    b_end = np.searchsorted(b_owner, base_of, side="right")
    m_len = b_end - b_start
    m_owner = np.repeat(members, m_len)
    idx = np.concatenate([np.arange(s, e) for s, e in zip(b_start, b_end)]) if len(members) else np.zeros(0, np.int64)
    src = b_elem[idx]
    keep = rng.random(len(idx)) >= np.repeat(f, m_len)
    repl = rng.integers(0, vocab, size=len(idx), dtype=np.int64)
    m_el = np.where(keep, src, repl)
    m_key = np.unique(m_owner.astype(np.int64) * vocab + m_el)
    # drop replaced ids that collided with a kept element (unique already merged them)
    all_key = np.concatenate([key, m_key])
    all_key.sort()
    owner = all_key // vocab
    elems = (all_key - owner * vocab).astype(np.uint32)
    offsets = np.zeros(n_sets + 1, np.int64)
    np.cumsum(np.bincount(owner, minlength=n_sets), out=offsets[1:])
    return SetCollection(offsets, elems, group, is_base, vocab)


def sorted_uniform_ids(n_obj: int, count: int, rng) -> np.ndarray:
    """`count` ids uniform on [0, n_obj), returned sorted (repeats possible)."""
    if count <= 0:
        return np.zeros(0, np.uint32)
    g = rng.exponential(size=count + 1)
    c = np.cumsum(g)
    return np.minimum((c[:-1] / c[-1] * n_obj).astype(np.int64), n_obj - 1).astype(np.uint32)


def member_lists(n_lists, n_obj, len_lo_exp, len_hi_exp, related, member_frac=0.01, seed=SEED_BASE + 3,
                 queries=None):
    """Candidate lists of length floor(10^U(lo, hi)): a fraction `member_frac` from
    the query's related objects (``related(q)``), the rest sorted uniform ids.
    Returns (queries uint32, offsets int64, cand uint32)."""
    rng = _rng(seed)
    lens = np.floor(10.0 ** rng.uniform(len_lo_exp, len_hi_exp, size=n_lists)).astype(np.int64)
    if queries is None:
        queries = rng.integers(0, n_obj, size=n_lists).astype(np.uint32)
    offsets = np.zeros(n_lists + 1, np.int64)
    np.cumsum(lens, out=offsets[1:])
    cand = np.empty(int(offsets[-1]), np.uint32)
    for i in range(n_lists):
        L = int(lens[i])
        rel = np.asarray(related(int(queries[i])), dtype=np.int64)
        n_rel = min(len(rel), int(round(member_frac * L)))
        pick = rng.choice(rel, size=n_rel, replace=False) if n_rel else np.zeros(0, np.int64)
        c = np.concatenate([pick.astype(np.uint32), sorted_uniform_ids(n_obj, L - n_rel, rng)])
        c.sort()
        cand[offsets[i]:offsets[i + 1]] = c
    return queries, offsets, cand


__all__ += ["jaccard_sets_large", "sorted_uniform_ids", "member_lists"]
