"""The seeded workload generators: determinism, the distributions the
workloads name, and the structure they plant (CPU, no GPU).  The generators
hold none of the method's arithmetic; these tests check only the inputs."""
import math

import numpy as np

from synth import generators as G


def _jac(a, b):
    a, b = set(a.tolist()), set(b.tolist())
    return len(a & b) / len(a | b)


def test_jaccard_sets_determinism_sizes_and_groups():
    s1 = G.jaccard_sets(n_sets=2000, seed=G.SEED_BASE + 1)
    s2 = G.jaccard_sets(n_sets=2000, seed=G.SEED_BASE + 1)
    s3 = G.jaccard_sets(n_sets=2000, seed=G.SEED_BASE + 2)
    assert np.array_equal(s1.offsets, s2.offsets) and np.array_equal(s1.elems, s2.elems)
    assert not (len(s1.elems) == len(s3.elems) and np.array_equal(s1.elems, s3.elems))
    sizes = np.diff(s1.offsets)
    assert sizes.min() >= 1
    # lognormal(ln 60, 0.8): median 60, log-sd 0.8 (background sets)
    bg = sizes[s1.group < 0]
    assert 52 <= np.median(bg) <= 68
    assert 0.7 <= np.std(np.log(bg)) <= 0.9
    for i in range(s1.n):       # sorted, unique, inside the vocabulary
        r = s1.row(i)
        assert np.all(np.diff(r.astype(np.int64)) > 0) and r.max() < s1.vocab
    # 100 groups of a base and 4 members; J(base, member) = (1 - f)/(1 + f), f in [0.1, 0.4]
    groups = np.unique(s1.group[s1.group >= 0])
    assert len(groups) == 100
    for g in groups:
        mem = np.flatnonzero(s1.group == g)
        assert len(mem) == 5 and s1.is_base[mem].sum() == 1
        b = mem[s1.is_base[mem]][0]
        for m in mem[~s1.is_base[mem]]:
            j = _jac(s1.row(b), s1.row(m))
            assert (1 - 0.4) / (1 + 0.4) - 0.03 <= j <= (1 - 0.1) / (1 + 0.1) + 0.03, j


def test_tfidf_corpus_nnz_norms_and_duplicates():
    c1 = G.tfidf_corpus(n_docs=3000, dim=1 << 20, seed=G.SEED_BASE + 21)
    c2 = G.tfidf_corpus(n_docs=3000, dim=1 << 20, seed=G.SEED_BASE + 21)
    assert np.array_equal(c1.indices, c2.indices) and np.array_equal(c1.values, c2.values)
    nnz = np.diff(c1.offsets)
    # Poisson(100) distinct terms per row: mean 100, variance 100
    assert abs(nnz.mean() - 100) < 2 and 70 < nnz.var() < 130
    norms = np.array([np.linalg.norm(c1.values[c1.offsets[i]:c1.offsets[i + 1]].astype(np.float64))
                      for i in range(c1.n)])
    np.testing.assert_allclose(norms, 1.0, atol=1e-6)
    assert c1.indices.max() < c1.dim
    # 5% planted near-duplicates, each close to its source
    dups = np.flatnonzero(c1.dup_source >= 0)
    assert abs(len(dups) - 0.05 * c1.n) <= 0.01 * c1.n
    cos = []
    for d in dups[:50]:
        ia, va = c1.row(d)
        ib, vb = c1.row(int(c1.dup_source[d]))
        common, pa, pb = np.intersect1d(ia, ib, return_indices=True)
        cos.append(float(np.dot(va[pa].astype(np.float64), vb[pb].astype(np.float64))))
    assert np.median(cos) > 0.6


def test_dense_mixture_norms_and_cosines():
    m = G.dense_mixture(n=4000, d=256, n_comp=20, seed=G.SEED_BASE + 31)
    np.testing.assert_allclose(np.linalg.norm(m.x.astype(np.float64), axis=1), 1.0, atol=1e-6)
    assert np.all((m.sigma >= 0.02) & (m.sigma <= 0.06))
    # within a component cos ~ 1 / (1 + d sigma^2); between components ~ 0
    rng = np.random.default_rng(1)
    for c in range(5):
        idx = np.flatnonzero(m.comp == c)[:40]
        cs = m.x[idx].astype(np.float64) @ m.x[idx].astype(np.float64).T
        within = cs[np.triu_indices(len(idx), 1)].mean()
        want = 1.0 / (1.0 + 256 * m.sigma[c] ** 2)
        assert abs(within - want) < 0.05, (within, want)
    a = rng.integers(0, m.x.shape[0], 3000)
    b = rng.integers(0, m.x.shape[0], 3000)
    keep = m.comp[a] != m.comp[b]
    between = np.sum(m.x[a[keep]].astype(np.float64) * m.x[b[keep]].astype(np.float64), axis=1)
    assert abs(between.mean()) < 0.02 and between.std() < 0.1


def test_calibration_agreement_rates():
    n_pairs, n = 400, 2048
    s = np.linspace(0.05, 0.95, n_pairs)
    bits = G.calibration_bits(n_pairs, n, s, 5)
    agree = (bits[0::2] == bits[1::2]).mean(axis=1)
    assert np.all(np.abs(agree - s) < 5 * np.sqrt(s * (1 - s) / n) + 1e-9)
    mh = G.calibration_minhash(n_pairs, 256, s, 6)
    agree = (mh[0::2] == mh[1::2]).mean(axis=1)
    assert np.all(np.abs(agree - s) < 5 * np.sqrt(s * (1 - s) / 256) + 1e-9)


def test_band_candidates_structure():
    corpus = G.tfidf_corpus(n_docs=1500, dim=1 << 16, mean_nnz=40, dup_frac=0.1, seed=G.SEED_BASE + 41)
    x, y = G.sparse_band_candidates(corpus, n_bands=8, band_bits=4, seed=G.SEED_BASE + 42)
    x2, y2 = G.sparse_band_candidates(corpus, n_bands=8, band_bits=4, seed=G.SEED_BASE + 42)
    assert np.array_equal(x, x2) and np.array_equal(y, y2)
    assert np.all(x < y) and len(x) > 0
    pairs = x.astype(np.int64) * corpus.n + y
    assert len(np.unique(pairs)) == len(pairs)          # each pair once
    # every planted duplicate that the bands can see collides with its source
    # with high probability (16-band LSH at high similarity)
    dups = np.flatnonzero(corpus.dup_source >= 0)
    s = set(pairs.tolist())
    hit = [min(d, int(corpus.dup_source[d])) * corpus.n + max(d, int(corpus.dup_source[d])) in s for d in dups]
    assert np.mean(hit) > 0.8


def test_sparse_band_bits_match_the_banded_candidates():
    """The packed band bits hold the signs the candidate generator bands:
    every pair listed shares a band key under them, and every pair sharing a
    key is listed (brute force over all pairs of a small corpus)."""
    corpus = G.tfidf_corpus(n_docs=300, dim=1 << 14, mean_nnz=30, dup_frac=0.1, seed=G.SEED_BASE + 43)
    nb, bb = 6, 5
    words = G.sparse_band_bits(corpus, n_bands=nb, band_bits=bb, seed=G.SEED_BASE + 44)
    assert words.shape == (corpus.n, 1) and words.dtype == np.uint32
    bits = (words[:, :, None] >> np.arange(32, dtype=np.uint32)) & 1
    bits = bits.reshape(corpus.n, 32).astype(bool)
    assert not bits[:, nb * bb:].any()                  # padding past the last band is zero
    keys = np.stack([(bits[:, b * bb:(b + 1) * bb] << np.arange(bb)).sum(1) for b in range(nb)], 1)
    i, j = np.triu_indices(corpus.n, 1)
    share = (keys[i] == keys[j]).any(1)
    want = set((i[share].astype(np.int64) * corpus.n + j[share]).tolist())
    x, y = G.sparse_band_candidates(corpus, n_bands=nb, band_bits=bb, seed=G.SEED_BASE + 44)
    assert set((x.astype(np.int64) * corpus.n + y).tolist()) == want and len(x) == len(want)
