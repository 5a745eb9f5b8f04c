"""GPU parity of the batched persistent path (bayeslsh_verify_batched): many
query lists of uneven lengths, mixed measures and per-list thresholds in one
graph launch, against the oracle run list by list at the same k."""
import numpy as np
import pytest
import torch

import paper_1110_1328_amd as P
from oracle import reference as R
from synth import generators as G

from gpu_util import decode_result, up, sigs_tensor

pytestmark = pytest.mark.gpu
EPS, DELTA, GAMMA = 0.03, 0.05, 0.03


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    c = P.bayeslsh_create(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def workload():
    """Two signature sets and 300 lists (lengths 10^U(0, 3.6), some empty).
    Objects 2i and 2i+1 agree per hash with probability s_i, so a query's
    partner q^1 is a planted near-neighbour; lists mix it with random ids."""
    rng = np.random.default_rng(2024)
    nj, nc = 4000, 5000
    sj = G.calibration_minhash(nj // 2, 256, rng.uniform(0.0, 1.0, nj // 2), 71)
    sc = G.pack_bits(G.calibration_bits(nc // 2, 1024, rng.uniform(0.5, 1.0, nc // 2), 72))
    n_lists = 300
    meas = rng.integers(0, 2, n_lists).astype(np.int32)
    ts = rng.choice([0.5, 0.7, 0.9], n_lists)
    lens = np.floor(10 ** rng.uniform(0, 3.6, n_lists)).astype(np.int64)
    lens[[3, 50]] = 0
    queries = np.where(meas == 0, rng.integers(0, nj, n_lists), rng.integers(0, nc, n_lists)).astype(np.uint32)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cand = np.empty(offsets[-1], np.uint32)
    for i in range(n_lists):
        n_obj = nj if meas[i] == 0 else nc
        c = rng.integers(0, n_obj, lens[i])
        c[: max(1, lens[i] // 50)] = queries[i] ^ 1
        cand[offsets[i]:offsets[i + 1]] = np.sort(c)[: lens[i]] if lens[i] else c
    return dict(sj=sj, sc=sc, meas=meas, ts=ts, lens=lens, queries=queries, offsets=offsets, cand=cand, nj=nj, nc=nc)


def oracle_batched(w, k):
    """k: one value for both measures or (k_jaccard, k_cosine)."""
    kj, kc = (k, k) if isinstance(k, int) else k
    n = len(w["cand"])
    dec = np.zeros(n, np.uint8)
    lvl = np.zeros(n, np.int16)
    mm = np.zeros(n, np.int32)
    sh = np.full(n, np.nan)
    for i in range(len(w["lens"])):
        s, e = w["offsets"][i], w["offsets"][i + 1]
        if s == e:
            continue
        sig = w["sj"] if w["meas"][i] == 0 else w["sc"]
        k = kj if w["meas"][i] == 0 else kc
        L = (256 if w["meas"][i] == 0 else 1024) // k
        x = np.full(e - s, w["queries"][i], np.uint32)
        r = R.verify(x, w["cand"][s:e], int(w["meas"][i]), sig, k, L, float(w["ts"][i]), EPS, DELTA, GAMMA)
        dec[s:e], lvl[s:e], mm[s:e], sh[s:e] = r["decision"], r["level"], r["m"], r["shat"]
    return dict(decision=dec, level=lvl, m=mm, shat=sh)


PREFIX = "word-major + prefix array"


def cosine_sigs(w, layout):
    """The cosine signature set in a layout, or word-major slabs with a
    separate 16 B/object array of hashes 0..127 (layout PREFIX)."""
    if layout == PREFIX:
        S = sigs_tensor(w["sc"], P.COSINE, P.WORD_MAJOR)
        return P.Signatures(S.data, P.COSINE, P.WORD_MAJOR, S.n_obj, S.n_hashes,
                            prefix=up(np.ascontiguousarray(w["sc"][:, :4])))
    return sigs_tensor(w["sc"], P.COSINE, layout)


def run_batched(ctx, w, k, layout=P.WORD_MAJOR):
    lists = P.list_descs(w["meas"], w["ts"], w["queries"], w["offsets"][:-1], w["lens"])
    cand = up(w["cand"])
    n = len(w["cand"])
    res = P.make_result(n, n, m_debug=True)
    Sj, Sc = sigs_tensor(w["sj"], P.JACCARD, P.OBJECT_MAJOR), cosine_sigs(w, layout)
    kk = P.bayeslsh_verify_batched(ctx, lists, cand, Sj, Sc, EPS, DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)   # the signature tensors stay referenced until the work is done
    del Sj, Sc
    return kk, decode_result(res, n)


def check(got, want):
    np.testing.assert_array_equal(got["decision"], want["decision"])
    np.testing.assert_array_equal(got["level"], want["level"])
    np.testing.assert_array_equal(got["m"], want["m"])
    acc = np.flatnonzero((want["decision"] == 1) | (want["decision"] == 2))
    np.testing.assert_array_equal(got["acc_idx"], acc)
    np.testing.assert_allclose(got["acc_val"], want["shat"][acc], atol=1e-6)


@pytest.mark.parametrize("k", [16, 32, 64, (16, 64), (64, 16)])
def test_batched_matches_oracle(ctx, workload, k):
    """Every k (one per measure or a pair); word-major, object-major (read
    128 hashes per gather) and word-major with a prefix array for the cosine
    signatures; several in-register depths before the survivor queue."""
    print("batched k=%s" % (k,), flush=True)
    want = oracle_batched(workload, k)
    kp = (k, k) if isinstance(k, int) else k
    for layout in (P.WORD_MAJOR, P.OBJECT_MAJOR, PREFIX):
        for inreg in (1, 3, 64):
            P.bayeslsh_set_tuning(ctx, batch_inreg=inreg, batch_blocks_per_cu=2)
            kk, got = run_batched(ctx, workload, k, layout=layout)
            assert kk == kp
            check(got, want)
    P.bayeslsh_set_tuning(ctx)
    assert len(set(want["decision"].tolist())) == 3


@pytest.mark.parametrize("k", [16, 32, 64])
def test_batched_tile_shapes_match_oracle(ctx, workload, k):
    """Every phase-1 tile shape: SRP wave tiles of 128, 256 and 512 candidates
    (2, 4, 8 per lane), minhash tiles of 64 and 128 (1, 2 per lane), each with
    survivors queued after one level and with every level in registers; the
    output is the oracle's list by list."""
    print("batched tile shapes k=%d" % k, flush=True)
    want = oracle_batched(workload, k)
    try:
        for ts in (128, 256, 512):
            for tm in (64, 128):
                for inreg in (1, 64):
                    P.bayeslsh_set_tuning(ctx, batch_inreg=inreg, batch_blocks_per_cu=2, batch_srp_tile=ts,
                                          batch_mh_tile=tm)
                    _, got = run_batched(ctx, workload, k, layout=P.OBJECT_MAJOR if ts == 256 else P.WORD_MAJOR)
                    t = P.bayeslsh_get_tuning(ctx)
                    assert (t["last_batch_srp_tile"], t["last_batch_mh_tile"]) == (ts, tm)
                    check(got, want)
    finally:
        P.bayeslsh_set_tuning(ctx)


def test_batched_tile_shape_rejected(ctx):
    for kw in ({"batch_srp_tile": 64}, {"batch_srp_tile": 1024}, {"batch_mh_tile": 32}, {"batch_mh_tile": 256}):
        with pytest.raises(P.BayesLSHError) as e:
            P.bayeslsh_set_tuning(ctx, **kw)
        assert e.value.code == -1
    P.bayeslsh_set_tuning(ctx)


def test_batched_spill_overflow_and_layout(ctx, workload):
    """A survivor queue far too small: survivors that find it full keep going in
    registers; object-major cosine signatures give the same output."""
    print("batched spill overflow", flush=True)
    want = oracle_batched(workload, 32)
    P.bayeslsh_set_tuning(ctx, batch_inreg=1, batch_spill_cap=37)
    _, got = run_batched(ctx, workload, 32, layout=P.OBJECT_MAJOR)
    check(got, want)
    P.bayeslsh_set_tuning(ctx)


def test_batched_staging_overflow(ctx, workload):
    """One staging entry per slice: nearly every accepted pair takes the
    direct path into the list; the output is still the oracle's, for the
    batched path and the exhaustive batched comparator."""
    print("batched staging overflow", flush=True)
    want = oracle_batched(workload, 32)
    n_acc = int(((want["decision"] == 1) | (want["decision"] == 2)).sum())
    assert n_acc > 4 * 256
    P.bayeslsh_set_tuning(ctx, acc_stage_cap=256)
    try:
        _, got = run_batched(ctx, workload, 32, layout=P.OBJECT_MAJOR)
        check(got, want)
        lists = P.list_descs(workload["meas"], workload["ts"], workload["queries"], workload["offsets"][:-1],
                             workload["lens"])
        n = len(workload["cand"])
        res = P.make_result(n, n, m_debug=True)
        Sj = sigs_tensor(workload["sj"], P.JACCARD, P.OBJECT_MAJOR)
        Sc = sigs_tensor(workload["sc"], P.COSINE, P.OBJECT_MAJOR)
        P.bayeslsh_exhaustive_batched(ctx, lists, up(workload["cand"]), Sj, Sc, EPS, DELTA, GAMMA, (1, 1), 32, res)
        P.bayeslsh_sync(ctx)
        check(decode_result(res, n), want)
    finally:
        P.bayeslsh_set_tuning(ctx)


def test_batched_graph_replays(ctx, workload):
    """The captured graph replayed several times with eager work and syncs in
    between: every replay matches the oracle."""
    print("batched replays", flush=True)
    want = oracle_batched(workload, 32)
    for rep in range(3):
        _, got = run_batched(ctx, workload, 32)
        check(got, want)
        torch.cuda.synchronize()
        _ = (torch.arange(1000, device="cuda") * 2).sum().item()


def test_batched_autotune(ctx, workload):
    print("batched autotune", flush=True)
    kk, got = run_batched(ctx, workload, 0)
    assert kk[0] in (16, 32, 64) and kk[1] in (16, 32, 64)
    t = P.bayeslsh_get_tuning(ctx)
    assert (t["last_batch_k_jaccard"], t["last_batch_k_cosine"]) == kk and t["last_batch_inreg"] in (1, 2, 4, 64)
    assert t["last_batch_srp_tile"] in (128, 256, 512) and t["last_batch_mh_tile"] in (64, 128)
    check(got, oracle_batched(workload, kk))
    kk2, _ = run_batched(ctx, workload, 0)   # cached choice: same k
    assert kk2 == kk
    kk3, got3 = run_batched(ctx, workload, (32, 0))   # Jaccard fixed, cosine tuned
    assert kk3[0] == 32 and kk3[1] in (16, 32, 64)
    check(got3, oracle_batched(workload, kk3))


def test_batched_bad_query_and_invalid_lists(ctx, workload):
    w = dict(workload)
    w["queries"] = workload["queries"].copy()
    w["queries"][7] = 10 ** 9          # out of range for both sets
    lists = P.list_descs(w["meas"], w["ts"], w["queries"], w["offsets"][:-1], w["lens"])
    n = len(w["cand"])
    res = P.make_result(n, n)
    cand = up(w["cand"])
    Sj, Sc = sigs_tensor(w["sj"], P.JACCARD, P.OBJECT_MAJOR), sigs_tensor(w["sc"], P.COSINE, P.WORD_MAJOR)
    P.bayeslsh_verify_batched(ctx, lists, cand, Sj, Sc, EPS, DELTA, GAMMA, (1, 1), 32, res)
    with pytest.raises(P.BayesLSHError) as e:
        P.bayeslsh_sync(ctx)
    assert e.value.code == -5
    s, t = w["offsets"][7], w["offsets"][8]
    assert np.all(res.code[s:t].cpu().numpy() == 0xFF)
    bad = P.list_descs([0], [0.7], [0], [n - 1], [5])          # runs past the end
    with pytest.raises(P.BayesLSHError):
        P.bayeslsh_verify_batched(ctx, bad, up(w["cand"]), sigs_tensor(w["sj"], P.JACCARD, P.OBJECT_MAJOR), None,
                                  EPS, DELTA, GAMMA, (1, 1), 32, res)
    cos_only = P.list_descs([1], [0.7], [0], [0], [5])
    with pytest.raises(P.BayesLSHError):   # a cosine list without cosine signatures
        P.bayeslsh_verify_batched(ctx, cos_only, up(w["cand"]), sigs_tensor(w["sj"], P.JACCARD, P.OBJECT_MAJOR), None,
                                  EPS, DELTA, GAMMA, (1, 1), 32, res)


@pytest.mark.parametrize("k", [16, 32, 64, (16, 64)])
def test_exhaustive_batched_equals_batched(ctx, workload, k):
    print("exhaustive batched k=%s" % (k,), flush=True)
    w = workload
    want = oracle_batched(w, k)
    lists = P.list_descs(w["meas"], w["ts"], w["queries"], w["offsets"][:-1], w["lens"])
    n = len(w["cand"])
    res = P.make_result(n, n, m_debug=True)
    cand = up(w["cand"])
    Sj, Sc = sigs_tensor(w["sj"], P.JACCARD, P.OBJECT_MAJOR), sigs_tensor(w["sc"], P.COSINE, P.OBJECT_MAJOR)
    P.bayeslsh_exhaustive_batched(ctx, lists, cand, Sj, Sc, EPS, DELTA, GAMMA, (1, 1), k, res)
    P.bayeslsh_sync(ctx)
    check(decode_result(res, n), want)


def test_batched_extreme_thresholds(ctx, workload):
    """Per-list thresholds near both ends of each measure's range (and one in
    the middle) in one batch: every list equals the oracle at its own t."""
    print("batched extreme thresholds", flush=True)
    rng = np.random.default_rng(77)
    w = dict(workload)
    low = np.where(w["meas"] == 0, 0.05, 0.52)
    pick = rng.integers(0, 3, len(w["lens"]))
    w["ts"] = np.where(pick == 0, low, np.where(pick == 1, 0.99, 0.7))
    want = oracle_batched(w, 32)
    for layout in (P.OBJECT_MAJOR, PREFIX):
        kk, got = run_batched(ctx, w, 32, layout=layout)
        assert kk == (32, 32)
        check(got, want)
    assert len(set(want["decision"].tolist())) == 3
