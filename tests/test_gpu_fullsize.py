"""Parity at the benchmark's full sizes, in the launch configuration the bench
times, on seeded samples of the outputs that the oracle computes one by one.

- Dense estimation: 1M x 256 Gaussian-mixture vectors, 1024 SRP bits, GPU LSH
  banding 16 x 12 bits of an independent 192-bit projection (2.4e9 candidates)
  handed over as bucket tiles, Algorithm 1 at t = 0.8, eps = gamma = 0.03,
  delta = 0.05, k = 32.  A stratified sample of 2^21 candidates (their ids
  from the same banding listed as id pairs, numbered alike) against the
  oracle on the GPU's own signatures: decision, level, m and S_hat; the id-pair
  path gives the same codes for every candidate.
- Cosine Lite: 100,000 tf-idf documents, 128 SRP bits, 16-band x 10-bit GPU
  banding (80.7M candidates), Algorithm 2 at t = 0.7, eps = 0.03, k = 32,
  h = 128.  A stratified sample of 2^20 candidates against the oracle's
  Algorithm 2 on the GPU's signatures and its FP64 exact cosines.
- Batched: 4096 query lists (about 4.4e8 candidates) over the 1M-set minhash
  index and the dense SRP index (word-major slabs plus the prefix array), k and
  launch shapes autotuned.  A stratified sample of 2^20 candidates against the
  oracle at each measure's chosen k and each list's threshold.

The oracle takes the GPU's signature bits as input (signature generation is
checked separately under the sign-flip rule), so every sampled output is
compared exactly."""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from oracle import reference as R
from synth import generators as G

from gpu_util import csr_device, down, up

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = P.bayeslsh_create(0)
    yield c
    c.close()


def _sample(n, n_sample, seed):
    """One uniform draw from each of n_sample equal strata of [0, n)."""
    rng = np.random.default_rng(seed)
    stride = n // n_sample
    return np.arange(n_sample, dtype=np.int64) * stride + rng.integers(0, stride, n_sample)


def _gather_u32(t, idx):
    return down(t.view(torch.int32)[torch.from_numpy(idx).cuda()].view(torch.uint32))


def _results_at(res, idx, n):
    d = torch.from_numpy(idx).cuda()
    code = res.code[:n][d].cpu().numpy()
    m = res.m_debug[:n].view(torch.int16)[d].cpu().numpy().view(np.uint16).astype(np.int32)
    na = int(res.n_accepted.item())
    assert na <= res.acc_idx.numel()
    val = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    val[res.acc_idx[:na].view(torch.int64)] = res.acc_val[:na]
    return code, m, val[d].cpu().numpy()


def _check(code, m, val, want, val_key, tol):
    np.testing.assert_array_equal(code >> 6, want["decision"])
    np.testing.assert_array_equal(code & 63, want["level"])
    np.testing.assert_array_equal(m, want["m"])
    emit = np.isfinite(want[val_key]) & (want["accepted"] if "accepted" in want else True)
    np.testing.assert_array_equal(np.isfinite(val), emit)
    assert np.max(np.abs(val[emit] - want[val_key][emit]), initial=0.0) <= tol


def test_dense_estimation_full_size(ctx):
    print("full size: dense estimation, 1M objects", flush=True)
    t, eps, delta, gamma, k = 0.8, 0.03, 0.05, 0.03, 32
    mix = G.dense_mixture(seed=G.SEED_BASE + 4)
    n_obj = mix.x.shape[0]
    xd = up(mix.x)
    planes = up(G.gaussian_planes(256, 1024, G.SEED_BASE + 204))
    sig = torch.empty(n_obj * 32, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), planes, 1024, 0, P.OBJECT_MAJOR, sig)
    band = torch.empty(n_obj * 6, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), up(G.gaussian_planes(256, 192, G.SEED_BASE + 104)), 192, 0,
                        P.OBJECT_MAJOR, band)
    P.bayeslsh_sync(ctx)
    del xd, mix
    S_band = P.Signatures(band, P.COSINE, P.OBJECT_MAJOR, n_obj, 192)
    tl, nt, n, trunc = P.bayeslsh_band_tiles(ctx, S_band, 16, 12, 1 << 25)
    assert not trunc and n > 2_000_000_000
    S = P.Signatures(sig, P.COSINE, P.OBJECT_MAJOR, n_obj, 1024)
    res = P.make_result(n, 1 << 28, m_debug=True)
    P.bayeslsh_verify(ctx, P.tiles(tl, nt, n), S, t, eps, delta, gamma, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    cap = n + 1024
    xo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    yo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    _, _, n_p, trunc = P.bayeslsh_band_candidates(ctx, S_band, 16, 12, cap, x_out=xo, y_out=yo, order_tile=16)
    assert not trunc and n_p == n
    # every candidate: the id-pair path's codes equal the tiles'
    res_p = P.make_result(n, 1 << 28)
    P.bayeslsh_verify(ctx, P.pairs(xo[:n], yo[:n]), S, t, eps, delta, gamma, (1, 1), k, res_p)
    P.bayeslsh_sync(ctx)
    assert bool(torch.equal(res.code[:n], res_p.code[:n]))
    assert int(res.n_accepted.item()) == int(res_p.n_accepted.item())
    del res_p
    # a stratified sample against the oracle
    idx = _sample(n, 1 << 21, 4101)
    xs, ys = _gather_u32(xo, idx), _gather_u32(yo, idx)
    code, m, val = _results_at(res, idx, n)
    sig_h = down(sig).reshape(n_obj, 32)
    want = R.verify(xs, ys, P.COSINE, sig_h, k, 1024 // k, t, eps, delta, gamma)
    _check(code, m, val, want, "shat", 1e-6)
    assert (want["decision"] == 0).any() and (want["decision"] == 1).any() and (want["decision"] == 2).any()


def test_cosine_lite_full_size(ctx):
    print("full size: cosine Lite, 100k documents", flush=True)
    t, eps, h, k = 0.7, 0.03, 128, 32
    corpus = G.tfidf_corpus(seed=G.SEED_BASE + 2)
    vec = csr_device(corpus)
    sig = torch.empty(corpus.n * (h // 32), dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, vec, None, h, 0x5EED_1110_1328, P.OBJECT_MAJOR, sig)
    words = G.sparse_band_bits(corpus, n_bands=16, band_bits=10, seed=G.SEED_BASE + 102)
    S_band = P.Signatures(up(words.reshape(-1)), P.COSINE, P.OBJECT_MAJOR, corpus.n, words.shape[1] * 32)
    cap = 1 << 27
    xo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    yo = torch.empty(cap, dtype=torch.int32, device="cuda").view(torch.uint32)
    _, _, n, trunc = P.bayeslsh_band_candidates(ctx, S_band, 16, 10, cap, x_out=xo, y_out=yo, order_tile=16)
    assert not trunc and n > 80_000_000
    S = P.Signatures(sig, P.COSINE, P.OBJECT_MAJOR, corpus.n, h)
    res = P.make_result(n, 1 << 22, m_debug=True)
    P.bayeslsh_lite_verify(ctx, P.pairs(xo[:n], yo[:n]), S, vec, t, eps, (1, 1), h, k, res)
    P.bayeslsh_sync(ctx)
    idx = _sample(n, 1 << 20, 4102)
    xs, ys = _gather_u32(xo, idx), _gather_u32(yo, idx)
    code, m, val = _results_at(res, idx, n)
    sig_h = down(sig).reshape(corpus.n, h // 32)
    want = R.verify(xs, ys, P.COSINE, sig_h, k, h // k, t, eps, 0, 0, lite=True)
    want = R.lite_finish(want, lambda a, b: R.exact_cosine_csr(corpus.offsets, corpus.indices, corpus.values, a, b),
                         xs, ys, t)
    _check(code, m, val, want, "exact", 1e-6)
    assert (want["decision"] == 0).any() and (want["decision"] == 3).any() and want["accepted"].any()


def _related(labels):
    """related(q): the other objects with q's label (label < 0: none)."""
    order = np.argsort(labels, kind="stable")
    lab = labels[order]
    starts = np.searchsorted(lab, labels, side="left")
    ends = np.searchsorted(lab, labels, side="right")

    def related(q):
        if labels[q] < 0:
            return np.zeros(0, np.int64)
        m = order[starts[q]:ends[q]]
        return m[m != q]
    return related


def _dense_index(ctx):
    """The dense cosine index: 1M x 256 mixture vectors, 1024 SRP bits as
    word-major slabs plus the 128-bit prefix array (what the batched and
    serving paths read), and the same bits object-major for the oracle."""
    mix = G.dense_mixture(seed=G.SEED_BASE + 4)
    n_c = mix.x.shape[0]
    xd = up(mix.x)
    planes = G.gaussian_planes(256, 1024, G.SEED_BASE + 204)
    pfx = torch.empty(n_c * 4, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), up(np.ascontiguousarray(planes[:, :128])), 128, 0,
                        P.OBJECT_MAJOR, pfx)
    sig_wm = torch.empty(n_c * 32, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), up(planes), 1024, 0, P.WORD_MAJOR, sig_wm)
    sig_om = torch.empty(n_c * 32, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_srp_sigs(ctx, P.dense_vectors(xd), up(planes), 1024, 0, P.OBJECT_MAJOR, sig_om)
    P.bayeslsh_sync(ctx)
    del xd
    return mix, P.Signatures(sig_wm, P.COSINE, P.WORD_MAJOR, n_c, 1024, prefix=pfx), sig_om


def test_batched_full_size(ctx):
    """The batched workload (4096 lists, lengths 10^U(2,6), measure ~
    Bernoulli(1/2), t in {0.5, 0.7, 0.9}; 1M minhash sets and the 1M x 1024-bit
    SRP index as word-major slabs plus the 128-bit prefix array), k and the
    launch shapes autotuned as the bench runs it: a stratified sample of 2^20
    candidates against the oracle at the chosen k of each measure and the
    list's threshold (decision, level, m, S_hat)."""
    print("full size: batched, 4096 lists", flush=True)
    eps, delta, gamma = 0.03, 0.05, 0.03
    sets = G.jaccard_sets_large(seed=G.SEED_BASE + 5)
    a, b = G.minhash_coeffs(256, G.SEED_BASE + 205)
    sig_j = torch.empty(sets.n * 256, dtype=torch.int32, device="cuda").view(torch.uint32)
    P.bayeslsh_minhash_sigs(ctx, P.set_vectors(up(sets.offsets), up(sets.elems), sets.vocab), up(a), up(b), sig_j)
    S_j = P.Signatures(sig_j, P.JACCARD, P.OBJECT_MAJOR, sets.n, 256)
    mix, S_c, sig_om = _dense_index(ctx)
    n_c = mix.x.shape[0]
    n_lists = 4096
    rng = np.random.default_rng(G.SEED_BASE + 3)
    meas = rng.integers(0, 2, n_lists).astype(np.int32)
    ts = rng.choice([0.5, 0.7, 0.9], n_lists)
    qj, oj, cj = G.member_lists(int(np.sum(meas == 0)), sets.n, 2, 6, _related(sets.group), seed=G.SEED_BASE + 31)
    qc, oc, cc = G.member_lists(int(np.sum(meas == 1)), n_c, 2, 6, _related(mix.comp), seed=G.SEED_BASE + 32)
    cand = np.concatenate([cj, cc])
    query = np.empty(n_lists, np.uint32)
    offset = np.empty(n_lists, np.int64)
    length = np.empty(n_lists, np.int64)
    ij, ic = np.flatnonzero(meas == 0), np.flatnonzero(meas == 1)
    query[ij], offset[ij], length[ij] = qj, oj[:-1], np.diff(oj)
    query[ic], offset[ic], length[ic] = qc, oc[:-1] + len(cj), np.diff(oc)
    lists = P.list_descs(meas, ts, query, offset, length)
    n = len(cand)
    assert n > 400_000_000
    res = P.make_result(n, 1 << 24, m_debug=True)
    kk = P.bayeslsh_verify_batched(ctx, lists, up(cand), S_j, S_c, eps, delta, gamma, (1, 1), 0, res)
    P.bayeslsh_sync(ctx)
    idx = _sample(n, 1 << 20, 4103)
    code, m, val = _results_at(res, idx, n)
    # each sampled candidate's list: lists are stored by position (the Jaccard
    # lists first), so sort the list starts
    order = np.argsort(offset, kind="stable")
    li = order[np.searchsorted(offset[order], idx, side="right") - 1]
    assert np.all((offset[li] <= idx) & (idx < offset[li] + length[li]))
    sigs_h = {0: down(sig_j).reshape(sets.n, 256), 1: down(sig_om).reshape(n_c, 32)}
    n_hash = {0: 256, 1: 1024}
    checked = 0
    seen = set()
    for me in (0, 1):
        for t in (0.5, 0.7, 0.9):
            sel = np.flatnonzero((meas[li] == me) & (ts[li] == t))
            if not len(sel):
                continue
            k = int(kk[me])
            want = R.verify(query[li[sel]], cand[idx[sel]], me, sigs_h[me], k, n_hash[me] // k, t, eps, delta, gamma)
            _check(code[sel], m[sel], val[sel], want, "shat", 1e-6)
            checked += len(sel)
            seen.update(np.unique(want["decision"]).tolist())
    assert checked == len(idx)
    assert {0, 1, 2} <= seen


def test_serving_full_size(ctx):
    """The serving workload: 10,000 queries against the dense index, candidate
    counts 10^U(3,6) (about 1.4e9 candidates), t = 0.8, k = 32, all submitted
    at once to a server with a 2 GiB admission budget, 128 active requests and
    2^23-candidate batches.  For a stratified sample of 2^20 candidates: in its
    request's accepted list iff the oracle emits S_hat for it, with the same
    value to 1e-6."""
    print("full size: serving, 10000 queries", flush=True)
    t, eps, delta, gamma = 0.8, 0.03, 0.05, 0.03
    mix, S, sig_om = _dense_index(ctx)
    n_obj = mix.x.shape[0]
    nq = 10000
    rng = np.random.default_rng(G.SEED_BASE + 6)
    queries = rng.integers(0, n_obj, nq).astype(np.uint32)
    q, off, cand = G.member_lists(nq, n_obj, 3, 6, _related(mix.comp), seed=G.SEED_BASE + 61, queries=queries)
    total = int(off[-1])
    assert total > 1_000_000_000
    idx = _sample(total, 1 << 20, 4104)
    req = np.searchsorted(off, idx, side="right") - 1
    bounds = np.searchsorted(req, np.arange(nq + 1))
    got_acc = np.zeros(len(idx), bool)
    got_val = np.full(len(idx), np.nan, np.float32)
    srv = P.Server(ctx, S, mem_budget_bytes=2 << 30, max_active=128, k=32, max_batch_candidates=1 << 23)
    try:
        ids = [srv.submit(int(q[i]), cand[off[i]:off[i + 1]], t) for i in range(nq)]
        for i, rid in enumerate(ids):
            r = srv.wait(rid)
            assert r["status"] == 0 and r["n_candidates"] == off[i + 1] - off[i]
            srv.release(rid)
            acc = r["acc_idx"]
            assert np.all(np.diff(acc) > 0) and (len(acc) == 0 or acc[-1] < r["n_candidates"])
            lo, hi = bounds[i], bounds[i + 1]
            local = idx[lo:hi] - off[i]
            pos = np.minimum(np.searchsorted(acc, local), max(len(acc) - 1, 0))
            hit = (acc[pos] == local) if len(acc) else np.zeros(hi - lo, bool)
            got_acc[lo:hi] = hit
            got_val[lo:hi][hit] = r["acc_val"][pos[hit]]
    finally:
        srv.close()
    want = R.verify(q[req], cand[idx], P.COSINE, down(sig_om).reshape(n_obj, 32), 32, 32, t, eps, delta, gamma)
    emit = np.isfinite(want["shat"])
    np.testing.assert_array_equal(got_acc, emit)
    assert np.max(np.abs(got_val[emit] - want["shat"][emit]), initial=0.0) <= 1e-6
    assert emit.any() and not emit.all()
