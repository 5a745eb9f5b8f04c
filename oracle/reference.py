"""Oracle entry points (test infrastructure only; never imported by the product).

Algorithm 1 (BayesLSH) and Algorithm 2 (BayesLSH-Lite) run per candidate
pair exactly as the paper states them:

    n, m = 0, 0
    repeat
        m += agreements among hashes [n, n + k)      (k hashes at a time)
        n += k
        prune   if Pr[S >= t | M(m,n)] < epsilon
        stop    if Pr[|S - S_hat| < delta | M(m,n)] >= 1 - gamma   (Algorithm 1 only)

Readings where the paper is silent: the hash range of
each step is [n, n+k) (the printed sum has k+1 terms); Algorithm 1 has no hash
budget, so a pair still undecided after the last available hash is emitted
with its estimate ("accepted at n_max"); Algorithm 2 checks pruning at
n = k, 2k, ..., h and then computes the exact similarity, emitting the pair
iff it is strictly greater than t.

The large-input loops are in ``ref.c`` (plain C, one candidate at a time);
``verify_py`` is a pure-Python restatement for tiny inputs that evaluates the
posterior afresh at every step (no memo), used to pin the C loop.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import posterior as P
from .build import OUT as _LIB_PATH, build as _build

DEC_PRUNED, DEC_CONC, DEC_NMAX, DEC_LITE = 0, 1, 2, 3
KIND_PAIRS, KIND_LISTS, KIND_ALL = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build(force=False)
        L = C.CDLL(path)
        p = C.c_void_p
        i32, i64, u64 = C.c_int32, C.c_int64, C.c_uint64
        L.philox4x32_10.argtypes = [p, p, p]
        L.srp_gauss.argtypes = [u64, C.c_uint32, C.c_uint32]
        L.srp_gauss.restype = C.c_float
        L.srp_sparse_proj.argtypes = [p, p, p, p, i64, i32, u64, i32, p]
        L.q16_encode_array.argtypes = [p, i64, p]
        L.q16_decode_array.argtypes = [p, i64, p]
        L.minhash.argtypes = [p, p, p, i64, p, p, i32, p]
        L.verify.argtypes = [i32, p, p, i64, i64, i32, p, i32, i32, i32, i32, p, p, p, p, p]
        L.count_all.argtypes = [p, p, i64, i32, p, i32, i32, p]
        L.exact_cosine_csr.argtypes = [p, p, p, p, p, i64, p]
        L.exact_cosine_dense.argtypes = [p, i64, p, p, i64, p]
        L.exact_jaccard.argtypes = [p, p, p, p, i64, p]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# LSH families (Section 4.1 minhash, Section 4.2 sign random projections)
# --------------------------------------------------------------------------
MINHASH_P = 2147483647  # 2^31 - 1


def minhash_signature_py(elems, a, b):
    """sig_h = min over e in the set of (a_h e + b_h) mod (2^31 - 1); Python integers."""
    return [min((int(ah) * int(e) + int(bh)) % MINHASH_P for e in elems) for ah, bh in zip(a, b)]


def minhash_signatures(offsets, elems, a, b, rows=None) -> np.ndarray:
    offsets = _c(offsets, np.int64)
    n = len(offsets) - 1
    rows = np.arange(n, dtype=np.int64) if rows is None else _c(rows, np.int64)
    lens = offsets[rows + 1] - offsets[rows]
    if np.any(lens == 0):
        raise ValueError("minhash of an empty set is undefined")
    elems = _c(elems, np.uint32)
    a = _c(a, np.uint32)
    b = _c(b, np.uint32)
    out = np.empty((len(rows), len(a)), np.uint32)
    lib().minhash(_ptr(offsets), _ptr(elems), _ptr(rows), len(rows), _ptr(a), _ptr(b), len(a), _ptr(out))
    return out


def philox4x32_10(ctr, key):
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox4x32_10_py(ctr, key):
    """Pure-Python Philox-4x32-10 (Salmon et al., SC 2011)."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    c = [int(v) & 0xFFFFFFFF for v in ctr]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & 0xFFFFFFFF, (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k0, p1 & 0xFFFFFFFF, (p0 >> 32) ^ c[3] ^ k1, p0 & 0xFFFFFFFF]
    return c


def srp_gauss(seed: int, term: int, bit: int) -> float:
    return float(lib().srp_gauss(seed, term, bit))


def srp_sparse_projections(offsets, indices, values, n_bits, seed, rows, q16=False) -> np.ndarray:
    """r_b . x in FP64 for sparse rows (Section 4.2); q16: every plane entry
    taken through its 2-byte storage (Section 4.3) first."""
    offsets = _c(offsets, np.int64)
    indices = _c(indices, np.uint32)
    values = _c(values, np.float32)
    rows = _c(rows, np.int64)
    out = np.empty((len(rows), n_bits), np.float64)
    lib().srp_sparse_proj(_ptr(offsets), _ptr(indices), _ptr(values), _ptr(rows), len(rows), n_bits, seed,
                          int(bool(q16)), _ptr(out))
    return out


def q16_encode(x) -> np.ndarray:
    """2-byte code of Gaussian samples (Section 4.3): floor((x + 8) 2^16 / 16),
    saturating outside (-8, 8)."""
    x = _c(np.atleast_1d(x), np.float64)
    out = np.empty(len(x), np.uint16)
    lib().q16_encode_array(_ptr(x), len(x), _ptr(out))
    return out


def q16_decode(codes) -> np.ndarray:
    """The value a 2-byte code stands for: the midpoint of its interval."""
    c = _c(np.atleast_1d(codes), np.uint16)
    out = np.empty(len(c), np.float64)
    lib().q16_decode_array(_ptr(c), len(c), _ptr(out))
    return out


def srp_dense_projections(X, R, rows=None) -> np.ndarray:
    """r_b . x in FP64 for dense float32 rows X[rows] and planes R [d, n_bits]."""
    Xs = X if rows is None else X[rows]
    return Xs.astype(np.float64) @ R.astype(np.float64)


def bits_from_projections(proj: np.ndarray) -> np.ndarray:
    """h_b(x) = 1 iff r_b . x >= 0, packed LSB-first: hash b -> word b//32, bit b%32."""
    n, nb = proj.shape
    if nb % 32:
        raise ValueError("number of hashes must be a multiple of 32")
    out = np.zeros((n, nb // 32), np.uint32)
    for b in range(nb):
        out[:, b // 32] |= (proj[:, b] >= 0).astype(np.uint32) << np.uint32(b % 32)
    return out


# --------------------------------------------------------------------------
# Algorithms 1 and 2
# --------------------------------------------------------------------------
def _agree_py(measure, sx, sy, i):
    if measure == P.JACCARD:
        return int(sx[i] == sy[i])
    return int(((int(sx[i // 32]) >> (i % 32)) & 1) == ((int(sy[i // 32]) >> (i % 32)) & 1))


def verify_py(x, y, measure, sig, k, n_levels, t, epsilon, delta, gamma, alpha=1.0, beta=1.0, lite=False):
    """Pure-Python Algorithm 1 / 2 for tiny inputs; the posterior is evaluated at every step."""
    out = []
    for px, py in zip(np.asarray(x).tolist(), np.asarray(y).tolist()):
        sx, sy = sig[px], sig[py]
        n = m = 0
        res = None
        for j in range(n_levels):
            m += sum(_agree_py(measure, sx, sy, i) for i in range(n, n + k))
            n += k
            if P.prune_prob(measure, m, n, t, alpha, beta) < epsilon:
                res = (DEC_PRUNED, j, m, math.nan)
                break
            s_hat = P.map_estimate(measure, m, n, alpha, beta)
            if not lite and P.concentration(measure, m, n, delta, alpha, beta) >= 1.0 - gamma:
                res = (DEC_CONC, j, m, s_hat)
                break
        if res is None:
            res = ((DEC_LITE if lite else DEC_NMAX), n_levels - 1, m,
                   math.nan if lite else P.map_estimate(measure, m, n, alpha, beta))
        out.append(res)
    dec = np.array([r[0] for r in out], np.uint8)
    lvl = np.array([r[1] for r in out], np.int16)
    mm = np.array([r[2] for r in out], np.int32)
    sh = np.array([r[3] for r in out], np.float64)
    return dict(decision=dec, level=lvl, m=mm, shat=sh)


def verify(x, y, measure, sig, k, n_levels, t, epsilon, delta, gamma, alpha=1.0, beta=1.0,
           lite=False, all_n=None):
    """Algorithm 1 (or 2 when lite) over explicit pairs, or over all pairs i<j of
    [0, all_n) in row-major order when ``all_n`` is given.

    ``sig`` is object-major: uint32 [n_obj, n_hashes] minhashes, or packed
    words [n_obj, n_bits/32] for sign random projections.
    Returns decision/level/m per pair and S_hat (NaN unless emitted by Algorithm 1).
    """
    sig = _c(sig, np.uint32)
    if sig.ndim != 2:
        raise ValueError("sig must be 2-D object-major")
    n_hashes = sig.shape[1] * (32 if measure == P.COSINE else 1)
    if n_levels * k > n_hashes:
        raise ValueError("not enough hashes for n_levels * k")
    memo = P.decision_memo(measure, float(t), float(epsilon), float(delta), float(gamma),
                           float(alpha), float(beta), int(k), int(n_levels), not lite)
    if all_n is None:
        x = _c(x, np.uint32)
        y = _c(y, np.uint32)
        n_pairs, kind = len(x), KIND_PAIRS
        if n_pairs and (int(x.max()) >= sig.shape[0] or int(y.max()) >= sig.shape[0]):
            raise ValueError("object id out of range")
    else:
        n_pairs, kind = all_n * (all_n - 1) // 2, KIND_ALL
        x = y = np.zeros(1, np.uint32)
    dec = np.empty(n_pairs, np.uint8)
    lvl = np.empty(n_pairs, np.int16)
    mm = np.empty(n_pairs, np.int32)
    survive = _c(memo["survive"], np.uint8)
    accept = _c(memo["accept"], np.uint8)
    lib().verify(kind, _ptr(x), _ptr(y), n_pairs, 0 if all_n is None else all_n, measure, _ptr(sig),
                 sig.shape[1], k, n_levels, int(lite), _ptr(survive), _ptr(accept), _ptr(dec), _ptr(lvl), _ptr(mm))
    sh = np.full(n_pairs, np.nan)
    emit = (dec == DEC_CONC) | (dec == DEC_NMAX)
    sh[emit] = memo["shat"][lvl[emit], mm[emit]]
    return dict(decision=dec, level=lvl, m=mm, shat=sh)


def all_pairs_xy(n: int):
    """Row-major enumeration of the pairs i < j of [0, n)."""
    i, j = np.triu_indices(n, 1)
    return i.astype(np.uint32), j.astype(np.uint32)


def lite_finish(res, exact_fn, x, y, t):
    """Second half of Algorithm 2: exact similarity on the survivors, emitted iff s > t."""
    idx = np.flatnonzero(res["decision"] == DEC_LITE)
    s = exact_fn(np.asarray(x)[idx], np.asarray(y)[idx]) if len(idx) else np.zeros(0)
    exact = np.full(len(res["decision"]), np.nan)
    exact[idx] = s
    res = dict(res)
    res["exact"] = exact
    res["accepted"] = np.zeros(len(res["decision"]), bool)
    res["accepted"][idx] = s > t
    return res


def counts_all(x, y, measure, sig, n_hashes):
    """m over the first n_hashes hashes for each pair (classical estimate m/n, Section 3)."""
    sig = _c(sig, np.uint32)
    x = _c(x, np.uint32)
    y = _c(y, np.uint32)
    out = np.empty(len(x), np.int32)
    lib().count_all(_ptr(x), _ptr(y), len(x), measure, _ptr(sig), sig.shape[1], n_hashes, _ptr(out))
    return out


def mle(x, y, measure, sig, n_hashes, t):
    """LSH Approx (Section 5.1): S_hat = m/n over n_hashes hashes (cosine: r2c(m/n)); emit iff S_hat >= t."""
    m = counts_all(x, y, measure, sig, n_hashes)
    r = m / float(n_hashes)
    s = r if measure == P.JACCARD else np.cos(np.pi * (1.0 - r))
    return dict(m=m, shat=s, accepted=s >= t)


# --------------------------------------------------------------------------
# Exact similarity
# --------------------------------------------------------------------------
def exact_cosine_csr(offsets, indices, values, x, y):
    offsets = _c(offsets, np.int64)
    indices = _c(indices, np.uint32)
    values = _c(values, np.float32)
    x = _c(x, np.uint32)
    y = _c(y, np.uint32)
    out = np.empty(len(x), np.float64)
    lib().exact_cosine_csr(_ptr(offsets), _ptr(indices), _ptr(values), _ptr(x), _ptr(y), len(x), _ptr(out))
    return out


def exact_cosine_dense(X, x, y):
    X = _c(X, np.float32)
    x = _c(x, np.uint32)
    y = _c(y, np.uint32)
    out = np.empty(len(x), np.float64)
    lib().exact_cosine_dense(_ptr(X), X.shape[1], _ptr(x), _ptr(y), len(x), _ptr(out))
    return out


def exact_jaccard(offsets, elems, x, y):
    offsets = _c(offsets, np.int64)
    elems = _c(elems, np.uint32)
    x = _c(x, np.uint32)
    y = _c(y, np.uint32)
    out = np.empty(len(x), np.float64)
    lib().exact_jaccard(_ptr(offsets), _ptr(elems), _ptr(x), _ptr(y), len(x), _ptr(out))
    return out


# ---------------------------------------------------------------------------
# LSH banding candidate generation (Section 2), plain Python
# ---------------------------------------------------------------------------
def band_keys(bits_words, n_bands, band_bits):
    """Key of band j of every object: its bits j*b .. j*b+b-1 (LSB-first packed
    words, bit h in word h // 32 at position h % 32), as an integer."""
    w = np.asarray(bits_words, dtype=np.uint64)
    n = w.shape[0]
    keys = np.zeros((n, n_bands), np.int64)
    for j in range(n_bands):
        for t in range(band_bits):
            h = j * band_bits + t
            bit = (w[:, h // 32] >> np.uint64(h % 32)) & np.uint64(1)
            keys[:, j] |= bit.astype(np.int64) << t
    return keys


def band_candidates(bits_words, n_bands, band_bits, max_bucket=0, tile=0):
    """Objects whose keys agree in some band are candidates; a pair is listed
    once, in the first band where its keys agree.  Order: band by band,
    buckets by increasing key, members by increasing id; the pairs (a, b),
    a < b, of a bucket's member positions in row-major order (tile = 0), or
    (tile = T > 0) by T x T tiles -- tile rows a // T, then tile columns
    b // T, then row-major inside the tile.  max_bucket > 0 keeps the first
    max_bucket members of each bucket."""
    keys = band_keys(bits_words, n_bands, band_bits)
    n = keys.shape[0]
    xs, ys = [], []
    for j in range(n_bands):
        buckets = {}
        for i in range(n):
            buckets.setdefault(int(keys[i, j]), []).append(i)
        for key in sorted(buckets):
            mem = buckets[key]
            if max_bucket:
                mem = mem[:max_bucket]
            pos = [(a, b) for a in range(len(mem)) for b in range(a + 1, len(mem))]
            if tile:
                pos.sort(key=lambda ab: (ab[0] // tile, ab[1] // tile, ab[0], ab[1]))
            for a, b in pos:
                x, y = mem[a], mem[b]
                if any(keys[x, jj] == keys[y, jj] for jj in range(j)):
                    continue
                xs.append(x)
                ys.append(y)
    return np.array(xs, np.uint32), np.array(ys, np.uint32)
