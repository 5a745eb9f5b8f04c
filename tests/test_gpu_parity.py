"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Decisions, decision levels and match counts are compared bit for bit; S_hat
and exact similarities within 1e-6 absolute.  Decision parity always runs on
identical signature inputs (drawn by the seeded generators, or minhash
signatures that are first shown to be bit-identical); SRP signature
generation is checked separately against the FP64 oracle with the sign-flip
rule (bits may differ only where |r . x| < 1e-5).
"""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from oracle import posterior as O
from oracle import reference as R
from synth import generators as G

from gpu_util import assert_same_as_oracle, csr_device, decode_result, down, sets_device, sigs_tensor, up

pytestmark = pytest.mark.gpu

T, EPS, DELTA, GAMMA = 0.7, 0.03, 0.05, 0.03


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    c = P.bayeslsh_create(0)
    yield c
    c.close()


def _flush(msg):
    print(msg, flush=True)


def run_verify(ctx, cand, sigs, t=T, k=32, prior=(1.0, 1.0), cap=None, m_debug=True):
    n = cand.count
    res = P.make_result(n, cap if cap is not None else max(16, n), m_debug=m_debug)
    P.bayeslsh_verify(ctx, cand, sigs, t, EPS, DELTA, GAMMA, prior, k, res)
    P.bayeslsh_sync(ctx)
    return res


# ---------------------------------------------------------------------------
# signatures
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_hashes", [256, 32, 100, 512, 1024])
def test_minhash_signatures_bit_exact(ctx, n_hashes):
    """Every hashes-per-lane variant (1, 2, 4, 8, 16), a count that is not a
    multiple of the wave (100), against the oracle bit for bit."""
    _flush("minhash sigs: 400 sets x %d hashes" % n_hashes)
    sets = G.jaccard_sets(n_sets=400, vocab=100_000, n_groups=20, seed=G.SEED_BASE + 11)
    a, b = G.minhash_coeffs(n_hashes, G.SEED_BASE + 12)
    out = torch.empty(sets.n * n_hashes, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_minhash_sigs(ctx, sets_device(sets), up(a), up(b), out)
    P.bayeslsh_sync(ctx)
    got = down(out).reshape(sets.n, n_hashes)
    want = R.minhash_signatures(sets.offsets, sets.elems, a, b)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n_bits,layout", [(2048, P.WORD_MAJOR), (128, P.OBJECT_MAJOR), (96, P.WORD_MAJOR),
                                           (512, P.OBJECT_MAJOR), (1024, P.WORD_MAJOR)])
def test_sparse_srp_signatures_flip_rule(ctx, n_bits, layout):
    _flush("sparse srp sigs: %d bits layout %d" % (n_bits, layout))
    corpus = G.tfidf_corpus(n_docs=300, dim=1 << 20, seed=G.SEED_BASE + 21)
    seed = 0x1234_5678_9ABC
    W = n_bits // 32
    out = torch.empty(corpus.n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, csr_device(corpus), None, n_bits, seed, layout, out)
    P.bayeslsh_sync(ctx)
    got = down(out).reshape((W, corpus.n) if layout == P.WORD_MAJOR else (corpus.n, W))
    if layout == P.WORD_MAJOR:
        got = got.T
    rows = np.arange(corpus.n, dtype=np.int64)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, n_bits, seed, rows)
    want = R.bits_from_projections(proj)
    diff = np.unpackbits((got ^ want).view(np.uint8), bitorder="little").reshape(corpus.n, n_bits).astype(bool)
    assert np.all(np.abs(proj[diff]) < 1e-5), np.abs(proj[diff]).max()
    assert diff.sum() <= max(1, 1e-6 * diff.size)


@pytest.mark.parametrize("n_bits,layout", [(2048, P.OBJECT_MAJOR), (96, P.WORD_MAJOR)])
def test_sparse_srp_plane_table_matches_on_the_fly(ctx, n_bits, layout):
    """With more nonzeros than twice the dimension the plane entries come from
    a table drawn once per term: bit-identical to drawing them per nonzero
    (the same CSR data declared with a dimension too large for a table), and
    the flip rule against the oracle."""
    _flush("sparse srp plane table: %d bits layout %d" % (n_bits, layout))
    corpus = G.tfidf_corpus(n_docs=1500, dim=1 << 12, mean_nnz=40, seed=G.SEED_BASE + 23)
    assert len(corpus.indices) > 2 * corpus.dim
    seed = 0x2222_3333_4444
    W = n_bits // 32
    off, idx, val = up(corpus.offsets), up(corpus.indices.astype(np.uint32)), up(corpus.values)
    outs = []
    for dim in (corpus.dim, 1 << 40):   # table; drawn per nonzero
        out = torch.empty(corpus.n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
        P.bayeslsh_srp_sigs(ctx, P.csr_vectors(off, idx, val, dim), None, n_bits, seed, layout, out)
        P.bayeslsh_sync(ctx)
        outs.append(down(out))
    np.testing.assert_array_equal(outs[0], outs[1])
    got = outs[0].reshape((W, corpus.n) if layout == P.WORD_MAJOR else (corpus.n, W))
    if layout == P.WORD_MAJOR:
        got = got.T
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, n_bits, seed,
                                    np.arange(corpus.n, dtype=np.int64))
    want = R.bits_from_projections(proj)
    diff = np.unpackbits((got ^ want).view(np.uint8), bitorder="little").reshape(corpus.n, n_bits).astype(bool)
    assert np.all(np.abs(proj[diff]) < 1e-5), np.abs(proj[diff]).max()
    assert diff.sum() <= max(1, 1e-6 * diff.size)


@pytest.mark.parametrize("d,n_bits,layout", [(256, 1024, P.WORD_MAJOR), (64, 64, P.OBJECT_MAJOR),
                                             (128, 256, P.OBJECT_MAJOR), (32, 32, P.OBJECT_MAJOR)])
def test_dense_srp_mfma_flip_rule(ctx, d, n_bits, layout):
    _flush("dense srp sigs: d=%d bits=%d" % (d, n_bits))
    mix = G.dense_mixture(n=5000 + 37, d=d, n_comp=50, seed=G.SEED_BASE + 31)   # ragged row tail
    Rm = G.gaussian_planes(d, n_bits, G.SEED_BASE + 32)
    W = n_bits // 32
    out = torch.empty(mix.x.shape[0] * W, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(up(mix.x)), up(Rm), n_bits, 0, layout, out)
    P.bayeslsh_sync(ctx)
    n = mix.x.shape[0]
    got = down(out).reshape((W, n) if layout == P.WORD_MAJOR else (n, W))
    if layout == P.WORD_MAJOR:
        got = got.T
    proj = R.srp_dense_projections(mix.x, Rm)
    want = R.bits_from_projections(proj)
    diff = np.unpackbits((got ^ want).view(np.uint8), bitorder="little").reshape(n, n_bits).astype(bool)
    assert np.all(np.abs(proj[diff]) < 1e-5), np.abs(proj[diff]).max()
    assert diff.sum() <= max(1, 1e-6 * diff.size)


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------
def _calib_pairs(measure, npairs, n_hashes, seed, lo=None):
    rng = np.random.default_rng(seed)
    s = rng.uniform(lo if lo is not None else (0.5 if measure else 0.0), 1.0, npairs)
    if measure == P.JACCARD:
        return G.calibration_minhash(npairs, n_hashes, s, seed)
    return G.pack_bits(G.calibration_bits(npairs, n_hashes, s, seed))


@pytest.mark.parametrize("measure", [P.JACCARD, P.COSINE])
@pytest.mark.parametrize("k", [16, 32, 64])
def test_verify_pairs_bit_exact(ctx, measure, k):
    """Pairs with similarities spread over the whole range; ragged count."""
    n_hashes = 256 if measure == P.JACCARD else 1024
    npairs = 20000 + 13
    _flush("verify pairs measure=%d k=%d" % (measure, k))
    sig = _calib_pairs(measure, npairs, n_hashes, 100 + k + measure)
    rng = np.random.default_rng(7)
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    y = x + 1
    # mix in unrelated pairs and self pairs
    sw = rng.random(npairs) < 0.3
    y[sw] = rng.integers(0, 2 * npairs, sw.sum()).astype(np.uint32)
    y[:5] = x[:5]
    L = n_hashes // k
    want = R.verify(x, y, measure, sig, k, L, T, EPS, DELTA, GAMMA)
    layouts = [P.OBJECT_MAJOR] if measure == P.JACCARD else [P.WORD_MAJOR, P.OBJECT_MAJOR]
    for layout in layouts:
        res = run_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, measure, layout), k=k)
        assert_same_as_oracle(decode_result(res, npairs), want)
    assert len(set(want["decision"].tolist())) == 3


# (n_hashes, k, t, epsilon, delta, gamma); t = None: near the low end for the measure
DEGENERATE = [
    (32, 32, 0.7, 0.03, 0.05, 0.03),       # a single level: n_max = k
    (64, 64, 0.8, 0.03, 0.05, 0.03),       # a single level at k = 64
    (256, 32, 0.99, 0.03, 0.05, 0.03),     # threshold near 1
    (256, 32, None, 0.03, 0.05, 0.03),     # threshold near the low end
    (256, 16, 0.7, 1e-4, 0.05, 1e-4),      # tiny epsilon and gamma
    (256, 64, 0.7, 0.5, 0.2, 0.5),         # large epsilon, delta and gamma
]


@pytest.mark.parametrize("measure", [P.JACCARD, P.COSINE])
@pytest.mark.parametrize("case", range(len(DEGENERATE)))
def test_degenerate_parameters(ctx, measure, case):
    """A single level, thresholds near the ends of the range and extreme
    epsilon / delta / gamma: decisions, levels and m bit-exact against the
    oracle, accepted estimates within 1e-6."""
    n_hashes, k, t, eps, delta, gamma = DEGENERATE[case]
    if t is None:
        t = 0.05 if measure == P.JACCARD else 0.52
    npairs = 3000 + 7
    _flush("degenerate measure=%d case=%d" % (measure, case))
    sig = _calib_pairs(measure, npairs, n_hashes, 300 + case + 10 * measure)
    rng = np.random.default_rng(8 + case)
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    y = x + 1
    sw = rng.random(npairs) < 0.3
    y[sw] = rng.integers(0, 2 * npairs, sw.sum()).astype(np.uint32)
    y[:3] = x[:3]
    want = R.verify(x, y, measure, sig, k, n_hashes // k, t, eps, delta, gamma)
    layouts = [P.OBJECT_MAJOR] if measure == P.JACCARD else [P.WORD_MAJOR, P.OBJECT_MAJOR]
    for layout in layouts:
        res = P.make_result(npairs, npairs, m_debug=True)
        P.bayeslsh_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, measure, layout), t, eps, delta, gamma,
                          (1.0, 1.0), k, res)
        P.bayeslsh_sync(ctx)
        assert_same_as_oracle(decode_result(res, npairs), want)


@pytest.mark.parametrize("k", [16, 32, 64])
@pytest.mark.parametrize("lite", [False, True])
def test_layouts_and_candidate_orders(ctx, k, lite):
    """Word-major slabs, object-major rows (16-byte prefix gathers),
    object-major rows at an unaligned offset (word gathers), and either of the
    last two with a separate prefix array give the oracle's output on
    bucket-major candidates and on random pairs."""
    _flush("layouts k=%d lite=%d" % (k, lite))
    n_obj, n_hashes = 6000, 1024
    sig = _calib_pairs(P.COSINE, n_obj // 2, n_hashes, 40 + k)
    rng = np.random.default_rng(k)
    xs, ys = [], []
    for _ in range(40):
        mem = np.sort(rng.choice(n_obj, rng.integers(20, 80), replace=False))
        i, j = np.triu_indices(len(mem), 1)
        xs.append(mem[i]); ys.append(mem[j])
    xb, yb = np.concatenate(xs).astype(np.uint32), np.concatenate(ys).astype(np.uint32)
    xr = rng.integers(0, n_obj, 30011).astype(np.uint32)
    yr = rng.integers(0, n_obj, 30011).astype(np.uint32)
    L = 4 if lite else n_hashes // k
    dense = np.ones((n_obj, 8), np.float32)
    dense[:, 0] = np.arange(n_obj)          # distinct rows: exact cosines < 1
    dvec = P.dense_vectors(up(dense))
    om = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    # object-major rows starting 4 bytes into the buffer: not 16-byte aligned
    buf = torch.zeros(om.data.numel() + 1, dtype=torch.int32, device="cuda")
    buf[1:] = om.data.reshape(-1).view(torch.int32)
    om_unaligned = P.Signatures(buf[1:].view(torch.uint32), P.COSINE, P.OBJECT_MAJOR, n_obj, n_hashes)
    # a separate 16 B/object prefix array (hashes 0..127) beside either layout
    pfx = up(np.ascontiguousarray(sig[:, :4]))
    wm = sigs_tensor(sig, P.COSINE, P.WORD_MAJOR)
    wm_pfx = P.Signatures(wm.data, P.COSINE, P.WORD_MAJOR, n_obj, n_hashes, prefix=pfx)
    om_unaligned_pfx = P.Signatures(om_unaligned.data, P.COSINE, P.OBJECT_MAJOR, n_obj, n_hashes, prefix=pfx)
    layouts = [wm, om, om_unaligned, wm_pfx, om_unaligned_pfx]
    for x, y in ((xb, yb), (xr, yr)):
        want = R.verify(x, y, P.COSINE, sig, k, L, T, EPS, DELTA, GAMMA, lite=lite)
        if lite:
            want = R.lite_finish(want, lambda p_, q_: R.exact_cosine_dense(dense, p_, q_), x, y, T)
        for S in layouts:
            res = P.make_result(len(x), len(x), m_debug=True)
            if lite:
                P.bayeslsh_lite_verify(ctx, P.pairs(up(x), up(y)), S, dvec, T, EPS, (1, 1), L * k, k, res)
            else:
                P.bayeslsh_verify(ctx, P.pairs(up(x), up(y)), S, T, EPS, DELTA, GAMMA, (1, 1), k, res)
            P.bayeslsh_sync(ctx)
            got = decode_result(res, len(x))
            assert_same_as_oracle(got, want, lite_exact=want["exact"] if lite else None)


@pytest.mark.parametrize("n_hashes,k", [(160, 32), (192, 64), (224, 16), (224, 32), (416, 32)])
def test_tail_on_rows_of_odd_word_counts(ctx, n_hashes, k):
    """Object-major SRP rows whose length is not a multiple of 4 words (160,
    192, 224, 416 hashes) beside a separate 128-bit prefix array: the levels
    past the prefix are read one word at a time, never past a row (the last
    object is in the candidate set, so its row ends the buffer), aligned and
    at a 4-byte offset; the oracle's decisions, levels, m and S_hat."""
    _flush("tail on %d-hash rows, k=%d" % (n_hashes, k))
    n_obj = 3001
    W = n_hashes // 32
    sig = _calib_pairs(P.COSINE, (n_obj + 1) // 2, n_hashes, 900 + n_hashes + k, lo=0.75)[:n_obj]
    rng = np.random.default_rng(n_hashes + k)
    x = np.concatenate([np.arange(0, n_obj - 1, 2), rng.integers(0, n_obj, 5000)]).astype(np.uint32)
    y = np.concatenate([np.arange(1, n_obj, 2), rng.integers(0, n_obj, 5000)]).astype(np.uint32)
    x[-1], y[-1] = n_obj - 1, n_obj - 2
    want = R.verify(x, y, P.COSINE, sig, k, n_hashes // k, T, EPS, DELTA, GAMMA)
    assert np.sum(want["level"] >= 128 // k) > 100   # the tail has work
    pfx = up(np.ascontiguousarray(sig[:, :4]))
    rows = up(np.ascontiguousarray(sig).reshape(-1))
    buf = torch.zeros(n_obj * W + 1, dtype=torch.int32, device="cuda")
    buf[1:] = rows.view(torch.int32)
    for data in (rows, buf[1:].view(torch.uint32)):
        S = P.Signatures(data, P.COSINE, P.OBJECT_MAJOR, n_obj, n_hashes, prefix=pfx)
        res = run_verify(ctx, P.pairs(up(x), up(y)), S, k=k)
        assert_same_as_oracle(decode_result(res, len(x)), want)


def test_verify_jaccard_workload_all_pairs(ctx):
    """The Jaccard workload at full size: 2000 sets, all 1,999,000 pairs, 256
    minhashes, k = 32, t = 0.7, Beta(1,1); explicit pairs give the same result."""
    _flush("jaccard workload: 2000 sets all pairs")
    sets = G.jaccard_sets()
    a, b = G.minhash_coeffs(256, G.SEED_BASE + 101)
    out = torch.empty(sets.n * 256, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_minhash_sigs(ctx, sets_device(sets), up(a), up(b), out)
    P.bayeslsh_sync(ctx)
    sig = R.minhash_signatures(sets.offsets, sets.elems, a, b)
    np.testing.assert_array_equal(down(out).reshape(sets.n, 256), sig)   # identical inputs from here on
    want = R.verify(None, None, P.JACCARD, sig, 32, 8, T, EPS, DELTA, GAMMA, all_n=sets.n)
    S = P.Signatures(out, P.JACCARD, P.OBJECT_MAJOR, sets.n, 256)
    res = run_verify(ctx, P.all_pairs(sets.n), S)
    got = decode_result(res, len(want["decision"]))
    assert_same_as_oracle(got, want)
    x, y = R.all_pairs_xy(sets.n)
    res2 = run_verify(ctx, P.pairs(up(x), up(y)), S)
    assert_same_as_oracle(decode_result(res2, len(x)), want)
    # planted near-duplicates are found
    assert got["n_accepted"] >= 50


def test_verify_query_lists(ctx):
    _flush("verify query lists")
    n_obj, n_hashes = 3000, 512
    sig = _calib_pairs(P.COSINE, n_obj // 2, n_hashes, 5)
    rng = np.random.default_rng(3)
    lens = np.array([0, 1, 5, 64, 0, 1000, 333, 2], np.int64)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    query = rng.integers(0, n_obj, len(lens)).astype(np.uint32)
    cand = rng.integers(0, n_obj, offsets[-1]).astype(np.uint32)
    cand[10:20] = query[3] ^ 1     # the query's calibration partner
    qx = np.repeat(query, lens)
    want = R.verify(qx, cand, P.COSINE, sig, 32, 16, 0.6, EPS, DELTA, GAMMA)
    n = int(offsets[-1])
    wm = sigs_tensor(sig, P.COSINE, P.WORD_MAJOR)
    # word-major (levels in registers), object-major rows (prefix kernel and
    # survivor tail), word-major with a prefix array (tail on slabs)
    layouts = [wm, sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR),
               P.Signatures(wm.data, P.COSINE, P.WORD_MAJOR, n_obj, n_hashes,
                            prefix=up(np.ascontiguousarray(sig[:, :4])))]
    for S in layouts:
        res = P.make_result(n, n, m_debug=True)
        P.bayeslsh_verify(ctx, P.query_lists(up(query), up(offsets), up(cand)), S, 0.6, EPS, DELTA, GAMMA, (1, 1),
                          32, res)
        P.bayeslsh_sync(ctx)
        assert_same_as_oracle(decode_result(res, n), want)


def test_verify_all_pairs_cosine_tail(ctx):
    """ALL_PAIRS (the candidate index decoded from the triangle) through the
    prefix kernel and the survivor tail, with a ragged last launch tile."""
    _flush("verify all pairs cosine (tail)")
    n_obj, n_hashes = 1203, 1024
    sig = _calib_pairs(P.COSINE, (n_obj + 1) // 2, n_hashes, 6)[:n_obj]
    want = R.verify(None, None, P.COSINE, sig, 32, n_hashes // 32, 0.7, EPS, DELTA, GAMMA, all_n=n_obj)
    n = n_obj * (n_obj - 1) // 2
    for layout in (P.OBJECT_MAJOR, P.WORD_MAJOR):
        res = P.make_result(n, n, m_debug=True)
        P.bayeslsh_verify(ctx, P.all_pairs(n_obj), sigs_tensor(sig, P.COSINE, layout), 0.7, EPS, DELTA, GAMMA,
                          (1, 1), 32, res)
        P.bayeslsh_sync(ctx)
        assert_same_as_oracle(decode_result(res, n), want)
    assert len(set(want["decision"].tolist())) == 3


def test_verify_nonuniform_prior(ctx):
    _flush("verify jaccard prior beta(2,3)")
    npairs = 5000
    sig = _calib_pairs(P.JACCARD, npairs, 128, 77)
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    want = R.verify(x, x + 1, P.JACCARD, sig, 32, 4, 0.5, EPS, DELTA, GAMMA, alpha=2.0, beta=3.0)
    res = run_verify(ctx, P.pairs(up(x), up(x + 1)), sigs_tensor(sig, P.JACCARD, P.OBJECT_MAJOR), t=0.5,
                     prior=(2.0, 3.0))
    assert_same_as_oracle(decode_result(res, npairs), want)


def test_n_max_below_stored_hashes(ctx):
    """A signature of 1024 bits verified with n_max = 256."""
    npairs = 3000
    sig = _calib_pairs(P.COSINE, npairs, 1024, 8)
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    want = R.verify(x, x + 1, P.COSINE, sig, 32, 8, T, EPS, DELTA, GAMMA)
    for layout in (P.WORD_MAJOR, P.OBJECT_MAJOR):
        res = run_verify(ctx, P.pairs(up(x), up(x + 1)), sigs_tensor(sig, P.COSINE, layout, n_max=256))
        assert_same_as_oracle(decode_result(res, npairs), want)


# ---------------------------------------------------------------------------
# Algorithm 2 and exact similarity
# ---------------------------------------------------------------------------
def test_lite_cosine_sparse(ctx):
    _flush("lite cosine sparse")
    corpus = G.tfidf_corpus(n_docs=3000, dim=1 << 16, mean_nnz=60, dup_frac=0.1, seed=G.SEED_BASE + 41)
    x, y = G.sparse_band_candidates(corpus, n_bands=8, band_bits=5, seed=G.SEED_BASE + 42)
    n = len(x)
    # signatures: oracle SRP of the corpus (an input to both sides)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, 256, 99,
                                    np.arange(corpus.n, dtype=np.int64))
    sig = R.bits_from_projections(proj)
    want = R.verify(x, y, P.COSINE, sig, 32, 4, T, EPS, 0, 0, lite=True)
    exact_fn = lambda a, b: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, a, b)
    want = R.lite_finish(want, exact_fn, x, y, T)
    res = P.make_result(n, n, m_debug=True)
    P.bayeslsh_lite_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, P.COSINE, P.WORD_MAJOR), csr_device(corpus),
                           T, EPS, (1, 1), 128, 32, res)
    P.bayeslsh_sync(ctx)
    got = decode_result(res, n)
    assert_same_as_oracle(got, want, lite_exact=want["exact"])
    assert got["n_accepted"] > 10 and (want["decision"] == R.DEC_LITE).sum() > got["n_accepted"]


@pytest.mark.parametrize("h,k", [(32, 32), (256, 32), (128, 64), (64, 16)])
def test_lite_hash_budgets(ctx, h, k):
    """Lite with one level before the exact similarity (h = k), with every
    stored hash (h = n_max) and other (h, k) pairs, on word-major slabs and on
    object-major rows (the 128-bit prefix path when h >= 128)."""
    _flush("lite budgets h=%d k=%d" % (h, k))
    corpus = G.tfidf_corpus(n_docs=2000, dim=1 << 16, mean_nnz=50, dup_frac=0.1, seed=G.SEED_BASE + 45)
    x, y = G.sparse_band_candidates(corpus, n_bands=8, band_bits=5, seed=G.SEED_BASE + 46)
    n = len(x)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, 256, 98,
                                    np.arange(corpus.n, dtype=np.int64))
    sig = R.bits_from_projections(proj)
    want = R.verify(x, y, P.COSINE, sig, k, h // k, T, EPS, 0, 0, lite=True)
    want = R.lite_finish(want, lambda a, b: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, a, b),
                         x, y, T)
    vec = csr_device(corpus)
    for layout in (P.WORD_MAJOR, P.OBJECT_MAJOR):
        res = P.make_result(n, n, m_debug=True)
        P.bayeslsh_lite_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, P.COSINE, layout), vec,
                               T, EPS, (1, 1), h, k, res)
        P.bayeslsh_sync(ctx)
        assert_same_as_oracle(decode_result(res, n), want, lite_exact=want["exact"])


def test_lite_jaccard_sets_and_dense_cosine(ctx):
    _flush("lite jaccard sets + dense cosine")
    sets = G.jaccard_sets(n_sets=600, vocab=20000, n_groups=40, seed=G.SEED_BASE + 51)
    a, b = G.minhash_coeffs(64, G.SEED_BASE + 52)
    sig = R.minhash_signatures(sets.offsets, sets.elems, a, b)
    x, y = R.all_pairs_xy(sets.n)
    want = R.lite_finish(R.verify(x, y, P.JACCARD, sig, 32, 2, 0.5, EPS, 0, 0, lite=True),
                         lambda p, q: R.exact_jaccard(sets.offsets, sets.elems, p, q), x, y, 0.5)
    res = P.make_result(len(x), len(x), m_debug=True)
    P.bayeslsh_lite_verify(ctx, P.all_pairs(sets.n), sigs_tensor(sig, P.JACCARD, P.OBJECT_MAJOR), sets_device(sets),
                           0.5, EPS, (1, 1), 64, 32, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, len(x)), want, lite_exact=want["exact"])
    # dense exact cosine
    mix = G.dense_mixture(n=1500, d=256, n_comp=30, seed=G.SEED_BASE + 53)
    Rm = G.gaussian_planes(256, 256, G.SEED_BASE + 54)
    sig2 = R.bits_from_projections(R.srp_dense_projections(mix.x, Rm))
    rng = np.random.default_rng(1)
    x2 = rng.integers(0, 1500, 40000).astype(np.uint32)
    y2 = rng.integers(0, 1500, 40000).astype(np.uint32)
    same = mix.comp[x2] == mix.comp[y2]
    assert same.sum() > 500
    want2 = R.lite_finish(R.verify(x2, y2, P.COSINE, sig2, 32, 4, 0.8, EPS, 0, 0, lite=True),
                          lambda p, q: R.exact_cosine_dense(mix.x, p, q), x2, y2, 0.8)
    res2 = P.make_result(len(x2), len(x2), m_debug=True)
    P.bayeslsh_lite_verify(ctx, P.pairs(up(x2), up(y2)), sigs_tensor(sig2, P.COSINE, P.WORD_MAJOR),
                           P.dense_vectors(up(mix.x)), 0.8, EPS, (1, 1), 128, 32, res2)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res2, len(x2)), want2, lite_exact=want2["exact"])


# ---------------------------------------------------------------------------
# exhaustive comparator
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("measure,k", [(P.JACCARD, 32), (P.COSINE, 32), (P.COSINE, 16), (P.COSINE, 64),
                                       (P.JACCARD, 64)])
def test_exhaustive_replay_equals_verify(ctx, measure, k):
    _flush("exhaustive replay measure=%d k=%d" % (measure, k))
    n_hashes = 256 if measure == P.JACCARD else 2048
    npairs = 10000 + 3
    sig = _calib_pairs(measure, npairs, n_hashes, 300 + k)
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    L = min(64, n_hashes // k)
    want = R.verify(x, x + 1, measure, sig, k, L, T, EPS, DELTA, GAMMA)
    S = sigs_tensor(sig, measure, P.OBJECT_MAJOR, n_max=L * k)
    res = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_exhaustive_verify(ctx, P.pairs(up(x), up(x + 1)), S, None, T, EPS, DELTA, GAMMA, (1, 1), k, 0,
                                 P.REPLAY, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, npairs), want)
    # classical estimate over all n_max hashes
    res = P.make_result(npairs, npairs, m_debug=True)
    P.bayeslsh_exhaustive_verify(ctx, P.pairs(up(x), up(x + 1)), S, None, T, EPS, DELTA, GAMMA, (1, 1), k, 0,
                                 P.MLE, res)
    P.bayeslsh_sync(ctx)
    got = decode_result(res, npairs)
    mle = R.mle(x, x + 1, measure, sig, L * k, T)
    np.testing.assert_array_equal(got["m"], mle["m"])
    acc = np.flatnonzero(mle["accepted"])
    np.testing.assert_array_equal(got["acc_idx"], acc)
    np.testing.assert_allclose(got["acc_val"], mle["shat"][acc], atol=1e-6)


def test_exhaustive_lite_replay(ctx):
    corpus = G.tfidf_corpus(n_docs=2000, dim=1 << 16, mean_nnz=50, dup_frac=0.1, seed=G.SEED_BASE + 61)
    x, y = G.sparse_band_candidates(corpus, n_bands=8, band_bits=4, seed=G.SEED_BASE + 62)
    proj = R.srp_sparse_projections(corpus.offsets, corpus.indices, corpus.values, 512, 5,
                                    np.arange(corpus.n, dtype=np.int64))
    sig = R.bits_from_projections(proj)
    want = R.lite_finish(R.verify(x, y, P.COSINE, sig, 32, 4, T, EPS, 0, 0, lite=True),
                         lambda p, q: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, p, q), x, y, T)
    res = P.make_result(len(x), len(x), m_debug=True)
    P.bayeslsh_exhaustive_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR),
                                 csr_device(corpus), T, EPS, 0.5, 0.5, (1, 1), 32, 128, P.REPLAY_LITE, res)
    P.bayeslsh_sync(ctx)
    assert_same_as_oracle(decode_result(res, len(x)), want, lite_exact=want["exact"])


def test_chunked_launches_past_two_to_the_28(ctx):
    """A candidate list longer than one verify launch (2^28 candidates) and
    than many comparator launches: the prefix verify with its survivor tail
    and the full-signature replay give the same codes and accepted set, and a
    seeded sample of positions (both sides of each launch boundary included)
    matches the oracle."""
    npairs, n_hashes, k = 4096, 1024, 32
    n = (1 << 28) + (1 << 24) + 77
    _flush("chunked launches n=%d" % n)
    sig = _calib_pairs(P.COSINE, npairs, n_hashes, 909)
    n_obj = 2 * npairs
    # candidate i: planted pair (2j, 2j+1) with j = i * 2654435761 mod 4096, or
    # every 7th an unrelated object as y
    i = torch.arange(n, dtype=torch.int64, device="cuda")
    x64 = 2 * ((i * 2654435761) % npairs)
    y64 = torch.where(i % 7 == 0, (i * 40503) % n_obj, x64 + 1)
    del i
    x = x64.to(torch.int32).view(torch.uint32)
    y = y64.to(torch.int32).view(torch.uint32)
    del x64, y64
    cand = P.pairs(x, y)
    wm_pfx = P.Signatures(sigs_tensor(sig, P.COSINE, P.WORD_MAJOR).data, P.COSINE, P.WORD_MAJOR, n_obj, n_hashes,
                          prefix=up(np.ascontiguousarray(sig[:, :4])))
    om = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    cap = n
    rv = P.make_result(n, cap)
    P.bayeslsh_verify(ctx, cand, wm_pfx, T, EPS, DELTA, GAMMA, (1, 1), k, rv)
    re = P.make_result(n, cap)
    P.bayeslsh_exhaustive_verify(ctx, cand, om, None, T, EPS, DELTA, GAMMA, (1, 1), k, 0, P.REPLAY, re)
    P.bayeslsh_sync(ctx)
    assert torch.equal(rv.code, re.code)
    na = int(rv.n_accepted.item())
    assert na == int(re.n_accepted.item()) and 0 < na <= cap
    ia, pa = torch.sort(rv.acc_idx[:na].view(torch.int64))
    ib, pb = torch.sort(re.acc_idx[:na].view(torch.int64))
    assert torch.equal(ia, ib)
    assert float((rv.acc_val[:na][pa] - re.acc_val[:na][pb]).abs().max()) <= 1e-6
    del ib, pb, re
    # seeded sample against the oracle
    rng = np.random.default_rng(910)
    edges = np.array([(1 << 24) * c + d for c in range(1, 17) for d in (-1, 0)] + [(1 << 28) - 1, 1 << 28, n - 1])
    pos = np.unique(np.concatenate([rng.integers(0, n, 20000), edges]))
    pos_t = torch.from_numpy(pos).cuda()
    xs = 2 * ((pos * 2654435761) % npairs)
    ys = np.where(pos % 7 == 0, (pos * 40503) % n_obj, xs + 1)
    xs, ys = xs.astype(np.uint32), ys.astype(np.uint32)
    want = R.verify(xs, ys, P.COSINE, sig, k, n_hashes // k, T, EPS, DELTA, GAMMA)
    code = rv.code[pos_t].cpu().numpy()
    np.testing.assert_array_equal(code >> 6, want["decision"])
    np.testing.assert_array_equal(code & 63, want["level"])
    hit = torch.searchsorted(ia, pos_t).clamp(max=na - 1)
    found = (ia[hit] == pos_t).cpu().numpy()
    acc = (want["decision"] == R.DEC_CONC) | (want["decision"] == R.DEC_NMAX)
    np.testing.assert_array_equal(found, acc)
    vals = rv.acc_val[:na][pa][hit].cpu().numpy()
    np.testing.assert_allclose(vals[acc], want["shat"][acc], atol=1e-6, rtol=0)


STAGE_SLICES = 256   # staging slices of the library: acc_stage_cap = 256 leaves one entry per slice


def test_accepted_staging_overflow(ctx):
    """With one staging entry per slice almost every accepted pair takes the
    direct path: Algorithm 1 (SRP with and without the survivor tail, minhash),
    Lite (SRP survivors queued for the exact kernel, minhash exact queue) and
    the comparator still give the oracle's output, and truncation still
    reports the true count."""
    _flush("staging overflow")
    P.bayeslsh_set_tuning(ctx, acc_stage_cap=STAGE_SLICES)
    try:
        npairs = 30000 + 7
        for measure, n_hashes in ((P.COSINE, 1024), (P.JACCARD, 256)):
            sig = _calib_pairs(measure, npairs, n_hashes, 77 + measure)
            x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
            y = x + 1
            L = n_hashes // 32
            want = R.verify(x, y, measure, sig, 32, L, T, EPS, DELTA, GAMMA)
            layouts = [P.OBJECT_MAJOR] if measure == P.JACCARD else [P.OBJECT_MAJOR, P.WORD_MAJOR]
            for layout in layouts:   # cosine object-major: prefix kernel + tail
                res = run_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, measure, layout))
                assert_same_as_oracle(decode_result(res, npairs), want)
            S = sigs_tensor(sig, measure, P.OBJECT_MAJOR, n_max=L * 32)
            res = P.make_result(npairs, npairs, m_debug=True)
            P.bayeslsh_exhaustive_verify(ctx, P.pairs(up(x), up(y)), S, None, T, EPS, DELTA, GAMMA, (1, 1), 32, 0,
                                         P.REPLAY, res)
            P.bayeslsh_sync(ctx)
            assert_same_as_oracle(decode_result(res, npairs), want)
            n_acc = int(((want["decision"] == R.DEC_CONC) | (want["decision"] == R.DEC_NMAX)).sum())
            assert n_acc > 10 * STAGE_SLICES
            res = P.make_result(npairs, n_acc // 3)
            P.bayeslsh_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, measure, P.OBJECT_MAJOR), T, EPS, DELTA,
                              GAMMA, (1, 1), 32, res)
            with pytest.raises(P.BayesLSHError) as e:
                P.bayeslsh_sync(ctx)
            assert e.value.code == -4
            assert int(res.n_accepted.item()) == n_acc
        # Lite: fused SRP exact and the minhash exact queue
        n_obj = 4000
        sig = _calib_pairs(P.COSINE, n_obj // 2, 512, 78, lo=0.6)
        dense = np.random.default_rng(79).standard_normal((n_obj, 16)).astype(np.float32)
        dense[1::2] = dense[0::2] + 0.05 * dense[1::2]
        x = np.arange(0, n_obj, 2, dtype=np.uint32)
        y = x + 1
        want = R.lite_finish(R.verify(x, y, P.COSINE, sig, 32, 4, 0.5, EPS, 0, 0, lite=True),
                             lambda p, q: R.exact_cosine_dense(dense, p, q), x, y, 0.5)
        assert want["accepted"].sum() > 10 * STAGE_SLICES // 8
        res = P.make_result(len(x), len(x), m_debug=True)
        P.bayeslsh_lite_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR),
                               P.dense_vectors(up(dense)), 0.5, EPS, (1, 1), 128, 32, res)
        P.bayeslsh_sync(ctx)
        assert_same_as_oracle(decode_result(res, len(x)), want, lite_exact=want["exact"])
        sets = G.jaccard_sets(n_sets=1200, vocab=20_000, n_groups=200, seed=G.SEED_BASE + 80)
        a, b = G.minhash_coeffs(128, G.SEED_BASE + 81)
        msig = R.minhash_signatures(sets.offsets, sets.elems, a, b)
        i, j = np.triu_indices(300, 1)
        x, y = i.astype(np.uint32), j.astype(np.uint32)
        want = R.lite_finish(R.verify(x, y, P.JACCARD, msig, 32, 2, 0.3, EPS, 0, 0, lite=True),
                             lambda p, q: R.exact_jaccard(sets.offsets, sets.elems, p, q), x, y, 0.3)
        res = P.make_result(len(x), len(x), m_debug=True)
        P.bayeslsh_lite_verify(ctx, P.pairs(up(x), up(y)), sigs_tensor(msig, P.JACCARD, P.OBJECT_MAJOR),
                               sets_device(sets), 0.3, EPS, (1, 1), 64, 32, res)
        P.bayeslsh_sync(ctx)
        assert_same_as_oracle(decode_result(res, len(x)), want, lite_exact=want["exact"])
    finally:
        P.bayeslsh_set_tuning(ctx)


# ---------------------------------------------------------------------------
# edge cases and error paths
# ---------------------------------------------------------------------------
def test_empty_and_tiny_inputs(ctx):
    sig = _calib_pairs(P.COSINE, 4, 256, 1)
    S = sigs_tensor(sig, P.COSINE, P.WORD_MAJOR)
    e = torch.empty(0, dtype=torch.int32, device="cuda").view(torch.uint32)
    res = P.make_result(1, 4)
    res.n_accepted.fill_(123)
    P.bayeslsh_verify(ctx, P.pairs(e, e), S, T, EPS, DELTA, GAMMA, (1, 1), 32, res)
    P.bayeslsh_sync(ctx)
    assert int(res.n_accepted.item()) == 0
    for n in (1, 2, 3, 5):
        x = np.zeros(n, np.uint32)
        y = np.arange(n, dtype=np.uint32) % 8
        want = R.verify(x, y, P.COSINE, sig, 32, 8, T, EPS, DELTA, GAMMA)
        got = decode_result(run_verify(ctx, P.pairs(up(x), up(y)), S), n)
        assert_same_as_oracle(got, want)
    res = P.make_result(1, 4)
    P.bayeslsh_verify(ctx, P.all_pairs(1), S, T, EPS, DELTA, GAMMA, (1, 1), 32, res)
    P.bayeslsh_sync(ctx)
    assert int(res.n_accepted.item()) == 0


def test_bad_object_ids_are_flagged(ctx):
    sig = _calib_pairs(P.COSINE, 50, 256, 2)
    S = sigs_tensor(sig, P.COSINE, P.WORD_MAJOR)
    x = np.arange(40, dtype=np.uint32)
    y = x + 1
    y[7] = 100          # out of range
    x[20] = 1 << 31
    res = P.make_result(40, 40)
    P.bayeslsh_verify(ctx, P.pairs(up(x), up(y)), S, T, EPS, DELTA, GAMMA, (1, 1), 32, res)
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_sync(ctx)
    assert e.value.code == -5
    code = res.code.cpu().numpy()
    assert code[7] == 0xFF and code[20] == 0xFF
    ok = np.setdiff1d(np.arange(40), [7, 20])
    want = R.verify(x[ok], y[ok], P.COSINE, sig, 32, 8, T, EPS, DELTA, GAMMA)
    np.testing.assert_array_equal(code[ok] >> 6, want["decision"])
    P.bayeslsh_sync(ctx)  # cleared


def test_truncation_reports_true_count(ctx):
    npairs = 4000
    sig = _calib_pairs(P.JACCARD, npairs, 128, 3, lo=0.9)
    x = np.arange(0, 2 * npairs, 2, dtype=np.uint32)
    want = R.verify(x, x + 1, P.JACCARD, sig, 32, 4, T, EPS, DELTA, GAMMA)
    n_acc = int(((want["decision"] == 1) | (want["decision"] == 2)).sum())
    assert n_acc > 100
    res = P.make_result(npairs, 100)
    P.bayeslsh_verify(ctx, P.pairs(up(x), up(x + 1)), sigs_tensor(sig, P.JACCARD, P.OBJECT_MAJOR), T, EPS, DELTA,
                      GAMMA, (1, 1), 32, res)
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_sync(ctx)
    assert e.value.code == -4
    assert int(res.n_accepted.item()) == n_acc
    idx = down(res.acc_idx).astype(np.int64)
    acc = set(np.flatnonzero((want["decision"] == 1) | (want["decision"] == 2)).tolist())
    assert set(idx.tolist()) <= acc


def test_invalid_arguments_rejected(ctx):
    sig = _calib_pairs(P.COSINE, 10, 256, 4)
    S = sigs_tensor(sig, P.COSINE, P.WORD_MAJOR)
    x = up(np.zeros(4, np.uint32))
    res = P.make_result(4, 4)
    bad = [dict(t=1.0), dict(k=24), dict(k=128), dict(prior=(2, 2)), dict(epsilon=0.0)]
    for kw in bad:
        a = dict(t=T, epsilon=EPS, k=32, prior=(1, 1))
        a.update(kw)
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_verify(ctx, P.pairs(x, x), S, a["t"], a["epsilon"], DELTA, GAMMA, a["prior"], a["k"], res)
        assert e.value.code == -1
    # prefix arrays: SRP only, 16-byte aligned, n_hashes >= 128
    pbuf = torch.zeros(4 * 10 + 1, dtype=torch.int32, device="cuda")
    bad_sigs = [P.Signatures(S.data, P.COSINE, P.WORD_MAJOR, 10, 256, prefix=pbuf[1:].view(torch.uint32)),
                P.Signatures(S.data, P.COSINE, P.WORD_MAJOR, 10, 96, prefix=pbuf[:40].view(torch.uint32)),
                P.Signatures(up(np.zeros((10, 128), np.uint32)), P.JACCARD, P.OBJECT_MAJOR, 10, 128,
                             prefix=pbuf[:40].view(torch.uint32))]
    for Sb in bad_sigs:
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_verify(ctx, P.pairs(x, x), Sb, T, EPS, DELTA, GAMMA, (1, 1), 32, res)
        assert e.value.code == -1
    S2 = sigs_tensor(sig, P.COSINE, P.WORD_MAJOR, n_max=96)     # not a multiple of k = 64
    with pytest.raises(P.BayesLSHError):
        P.bayeslsh_verify(ctx, P.pairs(x, x), S2, T, EPS, DELTA, GAMMA, (1, 1), 64, res)
    with pytest.raises(P.BayesLSHError):   # Lite budget not a multiple of k
        P.bayeslsh_lite_verify(ctx, P.pairs(x, x), S, P.dense_vectors(torch.zeros(10, 8, device="cuda")), T, EPS,
                               (1, 1), 48, 32, res)


def test_near_tie_parameters_refused(ctx):
    """Section 4.3's table decisions are unique only away from ties: epsilon
    placed exactly on the oracle's Pr[S >= t | M(m, n)] at (n, m) = (64, 45)
    (cosine, t = 0.8), or 1 - gamma on its concentration at (96, 90)
    (Jaccard, t = 0.7), is refused with BLSH_EINVAL naming (n, m) by
    Algorithm 1, Lite, the exhaustive comparator and the batched call, with
    nothing enqueued (the outputs keep their sentinel); nudged by 1e-6 the
    same calls run."""
    n = 64
    sig = _calib_pairs(P.COSINE, n // 2, 256, 14)
    S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
    x = up(np.arange(0, n, 2, dtype=np.uint32))
    y = up(np.arange(1, n, 2, dtype=np.uint32))
    cand = P.pairs(x, y)
    eps_tie = O.prune_prob(1, 45, 64, 0.8)
    dvec = P.dense_vectors(torch.ones(n, 8, device="cuda"))
    calls = {
        "verify": lambda r, e: P.bayeslsh_verify(ctx, cand, S, 0.8, e, DELTA, GAMMA, (1, 1), 32, r),
        "lite": lambda r, e: P.bayeslsh_lite_verify(ctx, cand, S, dvec, 0.8, e, (1, 1), 128, 32, r),
        "exhaustive": lambda r, e: P.bayeslsh_exhaustive_verify(ctx, cand, S, None, 0.8, e, DELTA, GAMMA, (1, 1),
                                                                32, 0, P.REPLAY, r),
    }
    for name, call in calls.items():
        res = P.make_result(n // 2, n)
        res.code.fill_(0xEE)
        with pytest.raises(P.BayesLSHError) as e:
            call(res, eps_tie)
        assert e.value.code == -1 and "n=64, m=45" in str(e.value), (name, str(e.value))
        P.bayeslsh_sync(ctx)
        assert bool((res.code == 0xEE).all()), name
        call(res, eps_tie + 1e-6)
        P.bayeslsh_sync(ctx)
        assert not bool((res.code == 0xEE).any()), name
    # the batched call, Jaccard list with 1 - gamma on a concentration value
    gamma_tie = 1.0 - O.concentration(0, 90, 96, DELTA)
    jsig = _calib_pairs(P.JACCARD, n // 2, 256, 15)
    SJ = sigs_tensor(jsig, P.JACCARD, P.OBJECT_MAJOR)
    lists = P.list_descs(np.array([0], np.int32), np.array([0.7]), np.array([0], np.uint32),
                         np.array([0], np.int64), np.array([n - 1], np.int64))
    cand_ids = up(np.arange(1, n, dtype=np.uint32))
    res = P.make_result(n - 1, n)
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_verify_batched(ctx, lists, cand_ids, SJ, None, EPS, DELTA, gamma_tie, (1, 1), (32, 32), res)
    assert e.value.code == -1 and "n=96, m=90" in str(e.value), str(e.value)
    P.bayeslsh_verify_batched(ctx, lists, cand_ids, SJ, None, EPS, DELTA, gamma_tie + 1e-6, (1, 1), (32, 32), res)
    P.bayeslsh_sync(ctx)


def test_exact_similarity_matches_oracle(ctx):
    """bayeslsh_exact_similarity: Jaccard of sets, cosine of CSR and dense rows,
    against the oracle's FP64 brute force; a bad id gives NaN and EBADID."""
    _flush("exact similarity")
    rng = np.random.default_rng(33)
    sets = G.jaccard_sets(n_sets=400, n_groups=20, seed=G.SEED_BASE + 41)
    corpus = G.tfidf_corpus(n_docs=3000, seed=G.SEED_BASE + 42)
    mix = G.dense_mixture(n=2000, d=96, n_comp=20, seed=G.SEED_BASE + 43)
    cases = [(sets_device(sets), sets.n, lambda x, y: R.exact_jaccard(sets.offsets, sets.elems, x, y)),
             (csr_device(corpus), corpus.n,
              lambda x, y: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, x, y)),
             (P.dense_vectors(up(mix.x)), mix.x.shape[0], lambda x, y: R.exact_cosine_dense(mix.x, x, y))]
    for vecs, n_obj, ref in cases:
        x = rng.integers(0, n_obj, 5003).astype(np.uint32)
        y = rng.integers(0, n_obj, 5003).astype(np.uint32)
        x[:10] = y[:10]                                    # self pairs: similarity 1
        got = down(P.bayeslsh_exact_similarity(ctx, P.pairs(up(x), up(y)), vecs))[:len(x)]
        P.bayeslsh_sync(ctx)
        np.testing.assert_allclose(got, ref(x, y), atol=1e-6, rtol=0)
        lq = up(np.array([0, 2], np.uint32))
        off = up(np.array([0, 3, 5], np.int64))
        cl = up(y[:5])
        got_l = down(P.bayeslsh_exact_similarity(ctx, P.query_lists(lq, off, cl, 5), vecs))[:5]
        P.bayeslsh_sync(ctx)
        np.testing.assert_allclose(got_l, ref(np.array([0, 0, 0, 2, 2], np.uint32), y[:5]), atol=1e-6, rtol=0)
    xb = up(np.array([0, sets.n], np.uint32))
    out = P.bayeslsh_exact_similarity(ctx, P.pairs(xb, up(np.array([1, 2], np.uint32))), sets_device(sets))
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_sync(ctx)
    assert e.value.code == -5
    o = down(out)
    assert np.isfinite(o[0]) and np.isnan(o[1])


def test_exact_similarity_long_rows(ctx):
    """Rows longer than one wave's LDS stage (512 entries): the longer row is
    searched in memory instead; CSR cosine and set Jaccard against the oracle."""
    _flush("exact similarity, long rows")
    rng = np.random.default_rng(34)
    corpus = G.tfidf_corpus(n_docs=300, dim=1 << 16, mean_nnz=800, dup_frac=0.1, seed=G.SEED_BASE + 44)
    lens = np.diff(corpus.offsets)
    assert (lens > 512).mean() > 0.9
    sets = G.jaccard_sets(n_sets=300, vocab=50000, median=900.0, n_groups=20, seed=G.SEED_BASE + 45)
    assert (np.diff(sets.offsets) > 512).mean() > 0.5
    cases = [(csr_device(corpus), corpus.n,
              lambda x, y: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, x, y)),
             (sets_device(sets), sets.n, lambda x, y: R.exact_jaccard(sets.offsets, sets.elems, x, y))]
    for vecs, n_obj, ref in cases:
        x = rng.integers(0, n_obj, 2003).astype(np.uint32)
        y = rng.integers(0, n_obj, 2003).astype(np.uint32)
        x[:10] = y[:10]
        got = down(P.bayeslsh_exact_similarity(ctx, P.pairs(up(x), up(y)), vecs))[:len(x)]
        P.bayeslsh_sync(ctx)
        np.testing.assert_allclose(got, ref(x, y), atol=1e-6, rtol=0)


def test_learned_prior_pipeline(ctx):
    """Section 4.1's learned prior end to end on the Jaccard workload: exact
    similarities of a random sample of candidate pairs on the GPU, the
    method-of-moments Beta fit, then Algorithm 1 over all 1,999,000 pairs with
    that (real-valued) prior -- against the oracle run at the oracle's own fit."""
    _flush("learned prior pipeline")
    sets = G.jaccard_sets()
    a, b = G.minhash_coeffs(256, G.SEED_BASE + 101)
    out = torch.empty(sets.n * 256, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_minhash_sigs(ctx, sets_device(sets), up(a), up(b), out)
    P.bayeslsh_sync(ctx)
    sig = R.minhash_signatures(sets.offsets, sets.elems, a, b)
    np.testing.assert_array_equal(down(out).reshape(sets.n, 256), sig)
    # candidates: all pairs; the sample: random positions among them
    xa, ya = R.all_pairs_xy(sets.n)
    pick = G.subsample_pairs(len(xa), 20000, G.SEED_BASE + 44)
    xs, ys = xa[pick], ya[pick]
    sims = down(P.bayeslsh_exact_similarity(ctx, P.pairs(up(xs), up(ys)), sets_device(sets)))[:len(xs)]
    P.bayeslsh_sync(ctx)
    want_sims = R.exact_jaccard(sets.offsets, sets.elems, xs, ys)
    np.testing.assert_allclose(sims, want_sims, atol=1e-12, rtol=0)
    (alpha, beta), fell = P.bayeslsh_fit_prior(sims)
    wa, wb, wfell = O.fit_beta_moments(want_sims)
    assert not fell and not wfell
    assert alpha == pytest.approx(wa, rel=1e-9) and beta == pytest.approx(wb, rel=1e-9)
    assert (alpha, beta) != (1.0, 1.0)
    want = R.verify(None, None, P.JACCARD, sig, 32, 8, T, EPS, DELTA, GAMMA, alpha=wa, beta=wb, all_n=sets.n)
    S = P.Signatures(out, P.JACCARD, P.OBJECT_MAJOR, sets.n, 256)
    res = run_verify(ctx, P.all_pairs(sets.n), S, prior=(alpha, beta))
    assert_same_as_oracle(decode_result(res, len(want["decision"])), want)


def test_fixed_workspace(ctx):
    """A context workspace reserved and fixed: calls that fit run without
    growing it (and give the output of a growing context); a call that needs
    more returns BLSH_ENOMEM before enqueuing anything (its outputs untouched);
    the sparse SRP with a workspace too small for its plane table draws the
    entries per nonzero, giving the table path's bits."""
    _flush("fixed workspace")
    c2 = P.bayeslsh_create(0)
    try:
        rng = np.random.default_rng(41)
        sig = G.pack_bits(G.calibration_bits(2000, 512, rng.uniform(0.5, 1.0, 2000), 42))
        S = sigs_tensor(sig, P.COSINE, P.OBJECT_MAJOR)
        n = 300_000
        x = rng.integers(0, 4000, n).astype(np.uint32)
        y = (x ^ 1).astype(np.uint32)
        y[::3] = rng.integers(0, 4000, len(y[::3]))
        cand = P.pairs(up(x), up(y))
        ref = P.make_result(n, n, m_debug=True)
        P.bayeslsh_verify(ctx, cand, S, 0.7, 0.03, 0.05, 0.03, (1, 1), 32, ref)
        P.bayeslsh_sync(ctx)
        want = decode_result(ref, n)
        # warm up, read the size, freeze it: the same call runs again without growing
        res = P.make_result(n, n, m_debug=True)
        P.bayeslsh_verify(c2, cand, S, 0.7, 0.03, 0.05, 0.03, (1, 1), 32, res)
        P.bayeslsh_sync(c2)
        size = P.bayeslsh_workspace_bytes(c2)
        assert size > 0
        P.bayeslsh_reserve_workspace(c2, size, fixed=True)
        res = P.make_result(n, n, m_debug=True)
        P.bayeslsh_verify(c2, cand, S, 0.7, 0.03, 0.05, 0.03, (1, 1), 32, res)
        P.bayeslsh_sync(c2)
        assert P.bayeslsh_workspace_bytes(c2) == size
        got = decode_result(res, n)
        np.testing.assert_array_equal(got["code"], want["code"])
        np.testing.assert_array_equal(got["acc_idx"], want["acc_idx"])
        np.testing.assert_array_equal(got["acc_val"], want["acc_val"])
        # a call that needs more than the fixed size: refused, nothing written
        big = 40 * n
        xb = np.resize(x, big)
        yb = np.resize(y, big)
        res_b = P.make_result(big, 16)
        res_b.code.fill_(0xEE)
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_verify(c2, P.pairs(up(xb), up(yb)), S, 0.7, 0.03, 0.05, 0.03, (1, 1), 32, res_b)
        assert e.value.code == -2 and "workspace" in str(e.value)
        P.bayeslsh_sync(c2)
        assert bool((res_b.code == 0xEE).all())
        assert P.bayeslsh_workspace_bytes(c2) == size
        # the sparse SRP: table path (growing context) vs per-nonzero (fixed, too small)
        corpus = G.tfidf_corpus(n_docs=1500, dim=1 << 12, mean_nnz=40, seed=G.SEED_BASE + 27)
        assert len(corpus.indices) > 2 * corpus.dim
        W = 2048 // 32
        outs = []
        for cc in (ctx, c2):
            out = torch.empty(corpus.n * W, dtype=torch.int32, device="cuda").view(torch.uint32)
            P.bayeslsh_srp_sigs(cc, csr_device(corpus), None, 2048, 0x77, P.OBJECT_MAJOR, out)
            P.bayeslsh_sync(cc)
            outs.append(down(out))
        np.testing.assert_array_equal(outs[0], outs[1])
        assert P.bayeslsh_workspace_bytes(c2) == size
        # unfixed: grows again
        P.bayeslsh_reserve_workspace(c2, 0, fixed=False)
        P.bayeslsh_verify(c2, P.pairs(up(xb), up(yb)), S, 0.7, 0.03, 0.05, 0.03, (1, 1), 32,
                          P.make_result(big, big))
        P.bayeslsh_sync(c2)
        assert P.bayeslsh_workspace_bytes(c2) > size
    finally:
        c2.close()
